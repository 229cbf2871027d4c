"""Pins of the CPU oracle against facts that do not come from the oracle:
textbook gate identities, tensor-contraction application, the closed form of
the QFT, unitarity, the HHL identity on exactly representable spectra,
special cases, library linear algebra and the paper's printed values.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads as W
from tests._ref import (apply_tensor, apply_ucry_tensor, cmat, inverse_gates,
                        max_abs_diff)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
I2 = np.eye(2)


# ---------------------------------------------------------------- gates ---
@pytest.mark.parametrize("theta", [0.0, 0.3, 1.7, -2.2, 5.9])
def test_rotation_gates_are_exponentials(theta):
    assert max_abs_diff(oracle.gate_matrix("ry", [theta]),
                        scipy.linalg.expm(-0.5j * theta * PY)) < 1e-15
    assert max_abs_diff(oracle.gate_matrix("rz", [theta]),
                        scipy.linalg.expm(-0.5j * theta * PZ)) < 1e-15
    # P(phi) equals RZ(phi) up to the global phase e^{i phi/2}
    assert max_abs_diff(oracle.gate_matrix("p", [theta]),
                        np.exp(0.5j * theta) * oracle.gate_matrix("rz", [theta])) < 1e-15


@pytest.mark.parametrize("seed", range(5))
def test_u3_is_zyz_product(seed):
    rng = np.random.default_rng(seed)
    th, ph, la = rng.uniform(0, 2 * np.pi, 3)
    zyz = (np.exp(0.5j * (ph + la)) * oracle.gate_matrix("rz", [ph])
           @ oracle.gate_matrix("ry", [th]) @ oracle.gate_matrix("rz", [la]))
    assert max_abs_diff(oracle.gate_matrix("u3", [th, ph, la]), zyz) < 1e-14


def test_fixed_gates():
    H = oracle.gate_matrix("h")
    assert max_abs_diff(H, (PX + PZ) / math.sqrt(2)) < 1e-15
    assert max_abs_diff(oracle.gate_matrix("x"), PX) == 0.0
    assert max_abs_diff(oracle.gate_matrix("u3", [np.pi / 2, 0, np.pi]), H) < 1e-15
    # CX = (I x H) CZ (I x H) with CZ = CP(pi), on qubit list (control, target)
    n = 2
    rng = np.random.default_rng(3)
    psi = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    via = apply_tensor(psi, n, [1], H)
    via = apply_tensor(via, n, [0, 1], oracle.gate_matrix("cp", [np.pi]))
    via = apply_tensor(via, n, [1], H)
    direct = apply_tensor(psi, n, [0, 1], oracle.gate_matrix("cx"))
    assert max_abs_diff(via, direct) < 1e-15
    # SWAP = CX(a,b) CX(b,a) CX(a,b)
    cx = oracle.gate_matrix("cx")
    s3 = apply_tensor(apply_tensor(apply_tensor(psi, n, [0, 1], cx), n, [1, 0], cx), n, [0, 1], cx)
    assert max_abs_diff(s3, apply_tensor(psi, n, [0, 1], oracle.gate_matrix("swap"))) < 1e-15
    # CP composes additively and is symmetric in its qubits
    assert max_abs_diff(oracle.gate_matrix("cp", [0.4]) @ oracle.gate_matrix("cp", [0.9]),
                        oracle.gate_matrix("cp", [1.3])) < 1e-15


def test_bell_state_golden():
    with open(os.path.join(GOLDEN, "bell_state.json")) as f:
        g = json.load(f)
    gates = [W.Gate(k, tuple(q), np.array(p, dtype=float)) for k, q, p in g["gates"]]
    out = oracle.apply_circuit(oracle.zero_state(g["n"]), g["n"], gates)
    want = np.array(g["amplitudes_re"]) + 1j * np.array(g["amplitudes_im"])
    assert max_abs_diff(out, want) < 1e-15


# ------------------------------------------------------- application ---
def _reference_apply(psi, n, g):
    if g.kind in oracle.KIND and g.kind not in ("dense", "cdense", "ucry"):
        return apply_tensor(psi, n, g.qubits, oracle.gate_matrix(g.kind, g.params))
    if g.kind == "dense":
        return apply_tensor(psi, n, g.qubits, cmat(g.params, len(g.qubits)))
    if g.kind == "cdense":
        return apply_tensor(psi, n, g.qubits[1:], cmat(g.params, len(g.qubits) - 1),
                            control=g.qubits[0])
    if g.kind == "ucry":
        return apply_ucry_tensor(psi, n, g.qubits[0], g.qubits[1:], g.params)
    raise ValueError(g.kind)


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (5, 3), (7, 4), (8, 5)])
def test_apply_matches_tensor_contraction(n, seed):
    gates = W.random_circuit(n, 40, seed, kmax=min(5, n))
    psi = W.random_state(n, seed)
    for g in gates:
        want = _reference_apply(psi, n, g)
        got = oracle.apply_circuit(psi, n, [g])
        assert max_abs_diff(got, want) < 1e-14, g.kind
        psi = want


@pytest.mark.parametrize("n,seed", [(6, 11), (10, 12)])
def test_norm_preserved_gate_by_gate(n, seed):
    psi = W.random_state(n, seed)
    for g in W.random_circuit(n, 60, seed, kmax=4):
        psi = oracle.apply_circuit(psi, n, [g])
        assert abs(np.vdot(psi, psi).real - 1.0) < 1e-13


@pytest.mark.parametrize("n,seed", [(5, 21), (9, 22)])
def test_mirror_returns_input(n, seed):
    gates = W.random_circuit(n, 80, seed, kmax=4)
    psi0 = W.random_state(n, seed)
    out = oracle.apply_circuit(oracle.apply_circuit(psi0, n, gates), n,
                               inverse_gates(gates))
    assert max_abs_diff(out, psi0) < 1e-13


# --------------------------------------------------------------- QFT ---
@pytest.mark.parametrize("m,q0,extra", [(1, 0, 0), (2, 1, 1), (3, 0, 2), (4, 2, 1), (6, 1, 0), (7, 0, 0)])
def test_qft_closed_form(m, q0, extra):
    n = q0 + m + extra
    M = 1 << m
    rng = np.random.default_rng(m)
    for x in sorted(set([0, 1, M - 1] + list(rng.integers(0, M, 3)))):
        other = (1 << q0) - 1 if q0 else 0     # some spectator bits set
        idx = (int(x) << q0) | other
        psi = np.zeros(1 << n, dtype=complex)
        psi[idx] = 1.0
        out = oracle.qft(psi, n, q0, m)
        e = np.zeros(M, dtype=complex)
        e[x] = 1.0
        closed = np.fft.ifft(e) * math.sqrt(M)   # 2^{-m/2} sum_y e^{+2 pi i x y / M}
        want = np.zeros(1 << n, dtype=complex)
        for y in range(M):
            want[(y << q0) | other] = closed[y]
        assert max_abs_diff(out, want) < 1e-14
    psi = W.random_state(n, m)
    back = oracle.qft(oracle.qft(psi, n, q0, m), n, q0, m, inverse=True)
    assert max_abs_diff(back, psi) < 1e-14


# ---------------------------------------------------- linear algebra ---
@pytest.mark.parametrize("N,seed", [(1, 0), (3, 1), (16, 2), (64, 3)])
def test_jacobi(N, seed):
    if N == 1:
        A = np.array([[2.5]])
    else:
        A, _ = W.dc_powerflow(N + 1, seed)
    lam, V, _ = oracle.jacobi(A)
    nA = np.linalg.norm(A, 2)
    assert np.linalg.norm(A @ V - V * lam) <= 1e-13 * nA
    assert np.linalg.norm(V.T @ V - np.eye(N)) <= 1e-14 * max(1, N)
    assert max_abs_diff(lam, np.linalg.eigvalsh(A)) <= 1e-13 * nA
    assert np.all(np.diff(lam) >= 0)


@pytest.mark.parametrize("N,seed", [(3, 0), (15, 1), (63, 2)])
def test_ge_solve(N, seed):
    A, b = W.dc_powerflow(N + 1, seed)
    x = oracle.ge_solve(A, b)
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b) * np.linalg.cond(A)
    assert max_abs_diff(x, np.linalg.solve(A, b)) <= 1e-12 * np.linalg.norm(x) * np.linalg.cond(A)


def test_qubit_count_table1():
    with open(os.path.join(GOLDEN, "table1_qubit_counts.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        rows = 2 * c["rows"] if c["dilated"] else c["rows"]
        nd, nq, nt = oracle.qubit_count(rows, c["kappa"], True)
        assert (nd, nq, nt) == (c["n_data"], c["n_qpe"], c["n_total"]), c["name"]


# --------------------------------------------------------------- HHL ---
@pytest.mark.parametrize("ns,m,seed", [(1, 4, 0), (2, 5, 1), (3, 6, 2), (4, 7, 3), (6, 8, 4)])
def test_hhl_exact_spectrum(ns, m, seed):
    """With eigenvalues on the clock grid, HHL returns A^{-1} b exactly."""
    A, b, t, _ = W.exact_spectrum_system(ns, m, seed)
    psi, x, xh, info = oracle.hhl_solve(A, b, m, t)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)
    assert abs(info["x_norm"] - np.linalg.norm(xs)) <= 1e-12 * np.linalg.norm(xs)
    bh = b / np.linalg.norm(b)
    p_expected = info["C"] ** 2 * np.linalg.norm(np.linalg.solve(A, bh)) ** 2
    assert abs(info["p1"] - p_expected) < 1e-12
    assert abs(info["p10"] - p_expected) < 1e-12
    n = info["n"]
    anc1 = np.abs(psi[1 << (n - 1):]) ** 2
    assert anc1.sum() - anc1[: 1 << ns].sum() < 1e-24 + 1e-12
    # 2m controlled 2^ns-term unitaries built from an eigen-decomposition:
    # rounding of order 2m * 2^ns * eps bounds the norm drift
    assert abs(np.vdot(psi, psi).real - 1) < 2 * m * (1 << ns) * 2.3e-16
    # The printed recovery |lambda_0| sqrt(P) does not give ||A^{-1} b_hat||;
    # sqrt(P) / lambda_0 does (C equals lambda_0 here).
    true_norm = np.linalg.norm(np.linalg.solve(A, bh))
    assert abs(math.sqrt(info["p1"]) / info["lambda_lo"] - true_norm) < 1e-10 * true_norm
    if abs(info["lambda_lo"] - 1) > 1e-3:
        assert abs(info["lambda_lo"] * math.sqrt(info["p1"]) - true_norm) > 1e-3 * true_norm


@pytest.mark.parametrize("N,lam", [(3, 2.0), (4, 0.5), (5, 7.25)])
def test_hhl_scaled_identity(N, lam):
    rng = np.random.default_rng(N)
    b = rng.standard_normal(N)
    A = lam * np.eye(N)
    psi, x, xh, info = oracle.hhl_solve(A, b, 4)
    assert max_abs_diff(x, b / lam) < 1e-13 * np.linalg.norm(b / lam) + 1e-15
    assert info["pad_leak"] < 1e-14
    assert info["max_imag"] < 1e-14


@pytest.mark.parametrize("seed", range(20))
def test_hhl_small_powerflow_fidelity(seed):
    """4-bus DC power flow, 4 clock qubits: fidelity to A^{-1} b (reported)."""
    A, b = W.dc_powerflow(4, seed)
    psi, x, xh, info = oracle.hhl_solve(A, b, 4)
    xs = oracle.ge_solve(A, b)
    fid = float(np.dot(xh, xs / np.linalg.norm(xs)) ** 2)
    # When kappa exceeds the clock range (2^m - 1) lambda_lo falls below one
    # clock step and the discretisation error dominates; still a fair answer.
    assert fid > (0.99 if info["kappa"] <= (1 << info["m"]) - 1 else 0.5)
    assert info["pad_leak"] < 1e-12
    assert abs(np.vdot(psi, psi).real - 1) < 1e-13
    # the smallest eigenvalue maps onto clock value j0 and the largest stays
    # in range (no wrap-around)
    scale = info["t"] * (1 << info["m"]) / (2 * math.pi)
    top = (1 << info["m"]) - 1
    if info["kappa"] <= top:
        assert abs(info["lambda_lo"] * scale - info["j0"]) < 1e-9
        assert info["lambda_hi"] * scale <= top + 1e-9
    else:
        assert abs(info["lambda_hi"] * scale - top) < 1e-9


def test_hhl_rejects_bad_inputs():
    A = np.array([[1.0, 2.0], [0.0, 1.0]])
    with pytest.raises(RuntimeError):
        oracle.hhl_solve(A, np.ones(2), 3)
    A = np.array([[1.0, 0.0], [0.0, -1.0]])
    with pytest.raises(RuntimeError):
        oracle.hhl_solve(A, np.ones(2), 3)
    with pytest.raises(RuntimeError):
        oracle.hhl_solve(np.eye(2), np.zeros(2), 3)


# ------------------------------------------ dilation and the sign qubit ---
@pytest.mark.parametrize("ns,m,seed", [(1, 4, 0), (2, 5, 1), (3, 6, 2), (4, 7, 3), (5, 8, 4)])
def test_hhl_signed_exact_spectrum(ns, m, seed):
    """Eigenvalues of both signs on the two's-complement clock grid: HHL with
    the sign qubit returns A^{-1} b exactly, signs included."""
    A, b, t, k = W.signed_spectrum_system(ns, m, seed)
    assert (k < 0).any() and (k > 0).any()
    psi, x, xh, info = oracle.hhl_solve(A, b, m, t, flags=oracle.HHL_SIGNED)
    xs = np.linalg.solve(A, b)
    assert info["sign_qubit"] == 1 and info["x_off"] == 0
    assert abs(info["lambda_lo"] - 0.25 * np.abs(k).min()) < 1e-12
    assert abs(info["lambda_hi"] - 0.25 * np.abs(k).max()) < 1e-12
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)
    bh = b / np.linalg.norm(b)
    p_expected = info["C"] ** 2 * np.linalg.norm(np.linalg.solve(A, bh)) ** 2
    assert abs(info["p10"] - p_expected) < 1e-12
    assert abs(info["p1"] - p_expected) < 1e-12
    assert info["max_imag"] < 1e-12
    assert abs(np.vdot(psi, psi).real - 1) < 2 * m * (1 << ns) * 2.3e-16


def test_hhl_signed_unsigned_clock_differ():
    """The same indefinite system without the sign qubit is refused, and a
    positive definite one solved with it still gives A^{-1} b."""
    A, b, t, k = W.signed_spectrum_system(2, 5, 7)
    with pytest.raises(RuntimeError):
        oracle.hhl_solve(A, b, 5, t)
    A, b, t, k = W.exact_spectrum_system(2, 4, 3)
    # magnitudes < 2^4 fit the 4 magnitude bits of a 5-bit signed clock
    _, x, _, info = oracle.hhl_solve(A, b, 5, t / 2, flags=oracle.HHL_SIGNED)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)


@pytest.mark.parametrize("N", [2, 5])
def test_hhl_negative_definite(N):
    """-A for a positive definite A: every eigenvalue negative, x = -x(A)."""
    rng = np.random.default_rng(N)
    lam = -0.5 * rng.integers(1, 8, size=N)      # -0.5 .. -3.5: grid of delta 0.5
    q = np.linalg.qr(rng.standard_normal((N, N)))[0]
    A = (q * lam) @ q.T
    A = 0.5 * (A + A.T)
    b = rng.standard_normal(N)
    m = 5
    t = 2 * math.pi / ((1 << m) * 0.5)
    _, x, _, info = oracle.hhl_solve(A, b, m, t, flags=oracle.HHL_SIGNED)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)
    _, x2, _, _ = oracle.hhl_solve(-A, b, m, t, flags=oracle.HHL_SIGNED)
    assert np.linalg.norm(x2 + xs) <= 1e-12 * np.linalg.norm(xs)


@pytest.mark.parametrize("N,seed", [(1, 0), (2, 1), (3, 2), (4, 3), (6, 4), (8, 5), (13, 6)])
def test_dilation_identity(N, seed):
    """Step 1c: H = [[0, A'], [A'^T, 0]] is symmetric, H [0; x] = [b_hat; 0]
    for the solution x of A x = b_hat, and its spectrum is +- the singular
    values of A' (those of A plus 1 for the pad)."""
    A, b = W.general_system(N, seed, kappa=30.0)
    H, bh, xo = oracle.hhl_system(A, b, oracle.HHL_DILATE)
    pa = 1 << max(0, math.ceil(math.log2(N)))
    assert H.shape == (2 * pa, 2 * pa) and xo == pa
    assert np.array_equal(H, H.T)
    x = np.linalg.solve(A, b / np.linalg.norm(b))
    v = np.zeros(2 * pa)
    v[pa:pa + N] = x
    rhs = np.zeros(2 * pa)
    rhs[:N] = b / np.linalg.norm(b)
    assert np.allclose(bh, rhs, rtol=0, atol=1e-15)
    assert np.linalg.norm(H @ v - rhs) < 1e-12 * np.linalg.norm(x) * 30
    sv = np.concatenate([np.linalg.svd(A, compute_uv=False), np.ones(pa - N)])
    ev = np.sort(np.linalg.eigvalsh(H))
    assert np.allclose(ev, np.sort(np.concatenate([sv, -sv])), rtol=0, atol=1e-12 * 30)
    # without the flag: the padded symmetric A (+) I
    S, bs = W.general_system(N, seed, kappa=30.0, symmetric=True)
    H2, bh2, xo2 = oracle.hhl_system(S, bs, 0)
    d = 1 << max(1, math.ceil(math.log2(N)))
    ref = np.eye(d)
    ref[:N, :N] = S
    assert xo2 == 0 and np.array_equal(H2, ref)


@pytest.mark.parametrize("N,m,seed", [(1, 4, 0), (2, 5, 1), (3, 6, 2), (4, 6, 3), (6, 7, 4), (8, 7, 5)])
def test_hhl_dilation_exact(N, m, seed):
    """A non-symmetric A whose singular values sit on the clock grid: the
    dilated solve returns A^{-1} b exactly from the second half of the
    system register, with nothing left in the first half."""
    A, b, t, k = W.nonsymmetric_exact_system(N, m, seed)
    assert np.abs(A - A.T).max() > 1e-3 or N == 1
    _, x, xh, info = oracle.hhl_solve(A, b, m, t, flags=oracle.HHL_DILATE)
    xs = np.linalg.solve(A, b)
    assert info["sign_qubit"] == 1
    assert info["x_off"] == 1 << max(0, math.ceil(math.log2(N)))
    assert info["ns"] == math.ceil(math.log2(N)) + 1
    sv = np.linalg.svd(A, compute_uv=False)
    assert abs(info["lambda_lo"] - sv.min()) < 1e-12 * sv.max()
    assert abs(info["lambda_hi"] - sv.max()) < 1e-12 * sv.max()
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)
    assert info["pad_leak"] < 1e-12
    assert info["max_imag"] < 1e-12


def test_hhl_dilation_symmetric_input():
    """Dilating a symmetric A gives the same x as solving it directly."""
    A, b, t, k = W.signed_spectrum_system(2, 6, 11)
    _, x1, _, _ = oracle.hhl_solve(A, b, 6, t, flags=oracle.HHL_SIGNED)
    _, x2, _, info = oracle.hhl_solve(A, b, 6, t, flags=oracle.HHL_DILATE)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x1 - xs) <= 1e-12 * np.linalg.norm(xs)
    assert np.linalg.norm(x2 - xs) <= 1e-12 * np.linalg.norm(xs)


@pytest.mark.parametrize("seed", range(6))
def test_hhl_dilation_converges_with_clock_bits(seed):
    """Off the grid, the dilated solve approaches A^{-1} b as clock qubits
    are added (phase-estimation error shrinks with resolution)."""
    A, b = W.general_system(4, seed, kappa=6.0)
    xs = np.linalg.solve(A, b)
    errs = []
    for m in (5, 8, 11):
        _, x, _, _ = oracle.hhl_solve(A, b, m, flags=oracle.HHL_DILATE,
                                      want_state=False)
        errs.append(np.linalg.norm(x - xs) / np.linalg.norm(xs))
    assert errs[2] < errs[0]
    assert errs[2] < 0.05


def test_hhl_signed_rejects_bad_inputs():
    A, b, t, k = W.signed_spectrum_system(1, 4, 0)
    with pytest.raises(RuntimeError):      # no magnitude bit left
        oracle.hhl_solve(A, b, 1, flags=oracle.HHL_SIGNED)
    with pytest.raises(RuntimeError):      # b reaches a zero eigenvalue
        oracle.hhl_solve(np.diag([1.0, 0.0]), np.ones(2), 4, flags=oracle.HHL_SIGNED)
    with pytest.raises(RuntimeError):      # unknown flag
        oracle.hhl_solve(np.eye(2), np.ones(2), 4, flags=8)
    # a zero eigenvalue b does not reach is harmless
    _, x, _, _ = oracle.hhl_solve(np.diag([2.0, 0.0]), np.array([1.0, 0.0]), 4,
                                  flags=oracle.HHL_SIGNED)
    assert abs(x[0] - 0.5) < 1e-12 and abs(x[1]) < 1e-12


@pytest.mark.parametrize("m", [2, 3, 5])
def test_hhl_signed_clock_range_ends(m):
    """The m-bit two's-complement clock spans -2^{m-1} .. 2^{m-1} - 1: an
    eigenvalue at exactly -2^{m-1} steps (phase -1/2) and one at +1 step are
    both inverted exactly, with their signs."""
    delta = 0.5
    lam = np.array([-(1 << (m - 1)) * delta, delta])
    q = np.linalg.qr(np.random.default_rng(m).standard_normal((2, 2)))[0]
    A = (q * lam) @ q.T
    A = 0.5 * (A + A.T)
    b = np.array([0.6, -0.8])
    t = 2 * math.pi / ((1 << m) * delta)
    _, x, _, info = oracle.hhl_solve(A, b, m, t, flags=oracle.HHL_SIGNED)
    xs = np.linalg.solve(A, b)
    assert info["j0"] == 1
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)


@pytest.mark.parametrize("seed", range(3))
def test_hhl_dilation_leak_accounting(seed):
    """Off the grid: x is read from the second half only, and pad_leak is
    the norm of every other postselected amplitude."""
    A, b = W.general_system(3, seed, kappa=5.0)
    psi, x, xh, info = oracle.hhl_solve(A, b, 6, flags=oracle.HHL_DILATE)
    n, xo = info["n"], info["x_off"]
    y = psi[1 << (n - 1):(1 << (n - 1)) + (1 << info["ns"])]
    keep = np.zeros(y.size, dtype=bool)
    keep[xo:xo + 3] = True
    assert abs(info["pad_leak"] - np.linalg.norm(y[~keep])) < 1e-14
    assert np.allclose(x, info["beta"] * y[keep].real / info["C"], rtol=0, atol=1e-14)
    assert abs(info["p10"] - np.vdot(y, y).real) < 1e-14


# ------------------------------------------------ Gauss-Seidel (step 1a) ---
@pytest.mark.parametrize("sym", [True, False])
@pytest.mark.parametrize("N,seed", [(1, 0), (3, 1), (5, 2), (13, 3), (29, 4)])
def test_gauss_seidel_system(N, seed, sym):
    """The preconditioned system is (M^{-1} A) x = M^{-1} b with M the lower
    triangle of A (numpy tril): M times the oracle's blocks gives back A and
    b, the solution is unchanged, and it is solved through the dilation.
    Symmetric (power flow) and non-symmetric inputs."""
    if N == 1:
        A, b = np.array([[2.5]]), np.array([1.5])
    elif sym:
        A, b = W.dc_powerflow(N + 1, seed)
    else:
        A, b = W.general_system(N, seed, kappa=10.0)
        A = A + 3.0 * np.eye(N)          # keep the diagonal away from zero
    info = oracle.hhl_params(A, b, 6, flags=oracle.HHL_GS)
    H, bh, xo = oracle.hhl_system(A, b, oracle.HHL_GS)
    pa = 1 << math.ceil(math.log2(N)) if N > 1 else 1
    assert xo == pa and H.shape == (2 * pa, 2 * pa)
    At = H[:N, pa:pa + N]
    assert np.array_equal(H[pa:pa + N, :N], At.T)
    M = np.tril(A)
    assert np.abs(M @ At - A).max() < 1e-12 * np.abs(A).max()
    bt = info["beta"] * bh[:N]
    assert np.abs(M @ bt - b).max() < 1e-12 * np.abs(b).max() * N
    x = np.linalg.solve(A, b)
    assert np.linalg.norm(At @ x - bt) < 1e-11 * np.linalg.norm(bt) * np.linalg.cond(A)
    assert info["sign_qubit"] == 1


@pytest.mark.parametrize("nbus,seed", [(14, 0), (30, 0), (30, 1), (64, 2)])
def test_gauss_seidel_condition_number(nbus, seed):
    """kappa of the preconditioned system is cond(M^{-1} A) (numpy SVD), and
    on the DC power-flow matrices it is lower than kappa(A), the effect
    Sec. IV reports for the 30-bus case (492.5 -> 109.3)."""
    A, b = W.dc_powerflow(nbus, seed)
    info = oracle.hhl_params(A, b, 8, flags=oracle.HHL_GS)
    kgs = np.linalg.cond(np.linalg.solve(np.tril(A), A))
    assert abs(info["kappa"] - kgs) < 1e-9 * kgs
    assert info["kappa"] < np.linalg.cond(A)


def test_gauss_seidel_hhl_converges_and_qubits():
    """The 30-bus shape: 29 unknowns -> 32 -> 64 (6 data qubits, Table I's
    30-bus* row); with enough clock qubits the preconditioned HHL solution
    approaches A^{-1} b."""
    A, b = W.dc_powerflow(30, 1)
    xs = np.linalg.solve(A, b)
    errs = []
    for m in (7, 9):
        _, x, _, info = oracle.hhl_solve(A, b, m, flags=oracle.HHL_GS, want_state=False)
        assert info["ns"] == 6 and info["x_off"] == 32
        errs.append(np.linalg.norm(x - xs) / np.linalg.norm(xs))
    assert errs[1] < errs[0] < 1.0


def test_gauss_seidel_rejects_zero_diagonal():
    A = np.array([[0.0, 1.0], [1.0, 2.0]])
    with pytest.raises(RuntimeError):
        oracle.hhl_solve(A, np.ones(2), 5, flags=oracle.HHL_GS)


# --------------------------------------------- Newton-Raphson power flow ---
def _two_bus(P, Q, x):
    return {"from": np.array([0], np.int32), "to": np.array([1], np.int32),
            "r": np.array([0.0]), "x": np.array([x]), "bsh": np.array([0.0]),
            "type": np.array([0, 2], np.int32), "p": np.array([0.0, -P]),
            "q": np.array([0.0, -Q]), "vset": np.array([1.0, 1.0])}


@pytest.mark.parametrize("P,Q,x", [(0.5, 0.2, 0.1), (1.2, 0.4, 0.2), (0.3, -0.1, 0.3)])
def test_pf_two_bus_closed_form(P, Q, x):
    """A load P + jQ fed over a lossless line jx from a 1.0 p.u. slack has
    V^4 + (2Qx - 1) V^2 + x^2 (P^2 + Q^2) = 0 (high-voltage root) and
    sin(-angle) = P x / V."""
    vm, va, info = oracle.pf_newton(_two_bus(P, Q, x), "ge")
    a = 1 - 2 * Q * x
    v2 = math.sqrt((a + math.sqrt(a * a - 4 * x * x * (P * P + Q * Q))) / 2)
    assert info["converged"]
    assert abs(vm[1] - v2) < 1e-10 and vm[0] == 1.0
    assert abs(va[1] + math.asin(P * x / v2)) < 1e-10


@pytest.mark.parametrize("nb,seed", [(5, 0), (14, 1), (30, 2)])
def test_pf_injections_are_complex_power(nb, seed):
    """P + jQ from the oracle's polar formulas equals V * conj(Y V) with Y
    assembled in complex numpy from the branch list."""
    c = W.ac_powerflow_case(nb, seed)
    rng = np.random.default_rng(seed)
    vm = rng.uniform(0.9, 1.1, nb)
    va = rng.uniform(-0.3, 0.3, nb)
    P, Q, F, J = oracle.pf_eval(c, vm, va)
    Y = np.zeros((nb, nb), dtype=complex)
    for f, t, r, x, b in zip(c["from"], c["to"], c["r"], c["x"], c["bsh"]):
        y = 1 / complex(r, x)
        Y[f, f] += y + 0.5j * b
        Y[t, t] += y + 0.5j * b
        Y[f, t] -= y
        Y[t, f] -= y
    V = vm * np.exp(1j * va)
    S = V * np.conj(Y @ V)
    assert np.abs(P - S.real).max() < 1e-12
    assert np.abs(Q - S.imag).max() < 1e-12


@pytest.mark.parametrize("nb,seed", [(5, 3), (14, 4)])
def test_pf_jacobian_is_derivative(nb, seed):
    """The Jacobian equals central finite differences of the mismatch."""
    c = W.ac_powerflow_case(nb, seed)
    rng = np.random.default_rng(seed)
    vm = rng.uniform(0.95, 1.05, nb)
    va = rng.uniform(-0.2, 0.2, nb)
    _, _, F0, J = oracle.pf_eval(c, vm, va)
    ty = c["type"]
    cols = [("a", i) for i in range(nb) if ty[i] != 0] + [("m", i) for i in range(nb) if ty[i] == 2]
    h = 1e-6
    for j, (kind, i) in enumerate(cols):
        vp, vq, ap, aq = vm.copy(), vm.copy(), va.copy(), va.copy()
        if kind == "a":
            ap[i] += h
            aq[i] -= h
        else:
            vp[i] += h
            vq[i] -= h
        Fp = oracle.pf_eval(c, vp, ap)[2]
        Fq = oracle.pf_eval(c, vq, aq)[2]
        # F = spec - injections, so dF/dx = -J
        fd = -(Fp - Fq) / (2 * h)
        assert np.abs(fd - J[:, j]).max() < 1e-7 * max(1.0, np.abs(J).max())


@pytest.mark.parametrize("nb,seed", [(14, 0), (30, 1)])
def test_pf_newton_quadratic_with_exact_solves(nb, seed):
    c = W.ac_powerflow_case(nb, seed)
    vm, va, info = oracle.pf_newton(c, "ge")
    h = info["history"]
    assert info["converged"] and info["mismatch"] < 1e-10
    # quadratic: once close, each mismatch is at most C times the square of the last
    tail = [(h[i], h[i + 1]) for i in range(len(h) - 1) if h[i] < 1e-2]
    assert tail and all(b <= 50 * a * a + 1e-13 for a, b in tail)


def test_pf_lossless_network_conserves_power():
    """With no resistance and no line charging, the injections sum to zero."""
    c = W.ac_powerflow_case(14, 5)
    c["r"] = np.zeros_like(c["r"])
    c["bsh"] = np.zeros_like(c["bsh"])
    vm, va, info = oracle.pf_newton(c, "ge")
    P, Q, F, J = oracle.pf_eval(c, vm, va)
    assert info["converged"] and abs(P.sum()) < 1e-10


@pytest.mark.parametrize("flags", [oracle.HHL_DILATE, oracle.HHL_GS])
def test_pf_newton_with_hhl_reaches_the_exact_solution(flags):
    """HHL as the inner solver (an inexact Newton step) converges to the
    same operating point as exact solves."""
    c = W.ac_powerflow_case(5, 0)
    v0, a0, _ = oracle.pf_newton(c, "ge")
    vm, va, info = oracle.pf_newton(c, "hhl", m=9, flags=flags, max_iter=30, tol=1e-9)
    assert info["converged"]
    assert np.abs(vm - v0).max() < 1e-8 and np.abs(va - a0).max() < 1e-8


def test_pf_rejects_bad_cases():
    c = _two_bus(0.5, 0.2, 0.1)
    c2 = dict(c, type=np.array([0, 0], np.int32))
    with pytest.raises(RuntimeError):
        oracle.pf_newton(c2, "ge")
    c3 = dict(c, x=np.array([0.0]))
    with pytest.raises(RuntimeError):
        oracle.pf_newton(c3, "ge")


@pytest.mark.parametrize("nb,seed", [(14, 6), (30, 7)])
def test_pf_solution_meets_the_specification(nb, seed):
    """At the converged point, checked with complex numpy arithmetic: |V| is
    the set point at slack and PV buses, P matches at every non-slack bus and
    Q at every PQ bus."""
    c = W.ac_powerflow_case(nb, seed, pv_frac=0.4)
    vm, va, info = oracle.pf_newton(c, "ge")
    assert info["converged"]
    Y = np.zeros((nb, nb), dtype=complex)
    for f, t, r, x, b in zip(c["from"], c["to"], c["r"], c["x"], c["bsh"]):
        y = 1 / complex(r, x)
        Y[f, f] += y + 0.5j * b
        Y[t, t] += y + 0.5j * b
        Y[f, t] -= y
        Y[t, f] -= y
    V = vm * np.exp(1j * va)
    S = V * np.conj(Y @ V)
    ty = c["type"]
    assert (ty == 1).any()
    assert np.abs(vm[ty != 2] - c["vset"][ty != 2]).max() < 1e-15
    assert abs(va[ty == 0][0]) < 1e-15
    assert np.abs(S.real[ty != 0] - c["p"][ty != 0]).max() < 1e-9
    assert np.abs(S.imag[ty == 2] - c["q"][ty == 2]).max() < 1e-9
