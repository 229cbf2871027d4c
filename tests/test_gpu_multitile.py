"""GPU parity of the multi-tile loops.

On a 33-qubit state every sweep kernel's wave walks many tiles (64 per wave
for a k = 4 dense gate), through the XCD-sliced tile range.  At the sizes the
oracle can check, a full-size grid gives each wave one tile, so these tests
bound the launch grid (``sv_debug_set_grid_cap``): with a bound of 8
workgroups (a multiple of the eight XCDs) the per-XCD slices are walked, with
3 the grid-wide stride.  The bound changes which wave takes which tile, not
any output element's arithmetic, so the full-state bars are those of the
unbounded runs: complex128 max |delta amplitude| <= 1e-12, complex64 <= 2e-5.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 2e-5}
CAPS = [3, 8]


def _hs():
    import paper_2402_08136_amd as hs
    return hs


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture
def grid_cap(request):
    hs = _hs()
    hs.sv_debug_set_grid_cap(request.param)
    yield request.param
    hs.sv_debug_set_grid_cap(0)


_ORACLE = {}


def _oracle_apply(key, psi0, n, gates):
    """oracle.apply_circuit, memoised per test case (both grid bounds and
    both dtypes check against the same FP64 result)."""
    if key not in _ORACLE:
        _ORACLE[key] = oracle.apply_circuit(psi0, n, gates)
    return _ORACLE[key]


def _run(n, gates, psi0, dtype, k=None):
    """Kernel-by-kernel launches (no cached graph), with the families used."""
    hs = _hs()
    c = hs.circuit_from_gates(n, gates)
    run = hs.fuse(c, k) if k else c
    s = hs.sv_create(n, dtype)
    s.set(psi0)
    _, fam = s.apply_timed(run)
    out = s.get()
    s.close()
    return out, {hs.KERNEL_FAMILY[int(f)] for f in fam}


# (name, targets for k = 1..5, families expected at complex128 / complex64).
# Every dense sweep family: registers (direct, complex64 pairs), the
# cross-lane butterfly (one or two targets inside a cache line; complex64 on
# pairs), the matrix cores (k = 5 with no target inside a line above the two
# lowest) and the LDS regroup (three targets inside a line, complex64 with
# bit 0 or two targets inside the line, k = 5 otherwise).
PATTERNS = {
    "high": [(9,), (7, 12), (6, 10, 15), (6, 8, 11, 17), (6, 7, 9, 13, 16)],
    "midline": [(4,), (3, 11), (5, 8, 14), (3, 4, 9, 16), (4, 5, 7, 12, 17)],
    "line1": [(1,), (2, 10), (1, 7, 13), (2, 6, 9, 15), (1, 6, 8, 12, 16)],
    "line2": [(0,), (0, 2), (1, 2, 11), (0, 2, 8, 14), (1, 2, 7, 10, 15)],
    "line3": [(2,), (0, 1), (0, 1, 2), (0, 1, 2, 9), (0, 1, 2, 6, 13)],
    "bit0": [(0,), (0, 7), (0, 5, 11), (0, 4, 9, 15), (0, 4, 6, 10, 16)],
}


@pytest.mark.parametrize("grid_cap", CAPS, indirect=True)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("pattern", list(PATTERNS))
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_dense_multitile(k, pattern, dtype, grid_cap):
    n = 18
    qs = list(PATTERNS[pattern][k - 1])
    rng = np.random.default_rng(4000 + 97 * k + len(pattern) + (7 if dtype == "c64" else 0))
    U = W.random_unitary(1 << k, rng)
    perm = rng.permutation(k)
    qs_list = [qs[i] for i in perm]
    g = W.Gate("dense", tuple(qs_list), np.ascontiguousarray(U).view(np.float64).ravel())
    _say(f"multitile dense n={n} targets={qs_list} dtype={dtype} cap={grid_cap}")
    psi0 = W.random_state(n, int(rng.integers(1 << 30)))
    want = oracle.apply_circuit(psi0, n, [g])
    got, fams = _run(n, [g], psi0, dtype)
    _say(f"  families {sorted(fams)}")
    assert fams and fams <= {"dense_direct", "dense_bfly", "dense_lds", "dense_mfma"}
    assert np.max(np.abs(got - want)) <= TOL[dtype]


@pytest.mark.parametrize("grid_cap", CAPS, indirect=True)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("pattern", list(PATTERNS))
@pytest.mark.parametrize("k", [4, 5])
def test_dense45_vector_form_multitile(k, pattern, dtype, grid_cap):
    """The vector kernels of 4- and 5-qubit gates (the matrix-core form
    switched off), over several tiles per wave."""
    hs = _hs()
    n = 18
    qs = list(PATTERNS[pattern][k - 1])
    rng = np.random.default_rng(7100 + len(pattern) + (7 if dtype == "c64" else 0))
    U = W.random_unitary(1 << k, rng)
    g = W.Gate("dense", tuple(qs), np.ascontiguousarray(U).view(np.float64).ravel())
    _say(f"multitile dense k={k} vector form n={n} targets={qs} dtype={dtype} cap={grid_cap}")
    psi0 = W.random_state(n, int(rng.integers(1 << 30)))
    want = oracle.apply_circuit(psi0, n, [g])
    hs.sv_debug_set_dense_mfma(False)
    try:
        got, fams = _run(n, [g], psi0, dtype)
    finally:
        hs.sv_debug_set_dense_mfma(True)
    _say(f"  families {sorted(fams)}")
    assert fams and fams <= {"dense_direct", "dense_bfly", "dense_lds"}
    assert np.max(np.abs(got - want)) <= TOL[dtype]


@pytest.mark.parametrize("grid_cap", CAPS, indirect=True)
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_bit0_pair_and_lds_forms_multitile(k, grid_cap):
    """complex64 gates with bit 0 the only target inside a line: the pair
    kernel and the LDS regroup it replaces, over several tiles per wave."""
    hs = _hs()
    n = 18
    qs = list(PATTERNS["bit0"][k - 1])
    rng = np.random.default_rng(8300 + k)
    U = W.random_unitary(1 << k, rng)
    g = W.Gate("dense", tuple(qs), np.ascontiguousarray(U).view(np.float64).ravel())
    psi0 = W.random_state(n, int(rng.integers(1 << 30)))
    want = oracle.apply_circuit(psi0, n, [g])
    for pair0 in (True, False):
        _say(f"multitile bit-0 gate n={n} targets={qs} pair kernel={pair0} cap={grid_cap}")
        hs.sv_debug_set_pair0(pair0)
        hs.sv_debug_set_dense_mfma(False)
        try:
            got, fams = _run(n, [g], psi0, "c64")
        finally:
            hs.sv_debug_set_pair0(True)
            hs.sv_debug_set_dense_mfma(True)
        _say(f"  families {sorted(fams)}")
        assert fams == ({"dense_direct"} if pair0 else {"dense_lds"})
        assert np.max(np.abs(got - want)) <= TOL["c64"]


@pytest.mark.parametrize("grid_cap", CAPS, indirect=True)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_random_circuit_multitile(k, dtype, grid_cap):
    """Fused random circuits (dense, diagonal, controlled and UCRY gates)."""
    n = 17
    gates = W.random_circuit(n, 60, 600 + k, kmax=5)
    psi0 = W.random_state(n, 600 + k)
    _say(f"multitile random circuit n={n} k={k} dtype={dtype} cap={grid_cap}")
    want = _oracle_apply(("rc", k), psi0, n, gates)
    got, fams = _run(n, gates, psi0, dtype, k)
    _say(f"  families {sorted(fams)}")
    assert np.max(np.abs(got - want)) <= TOL[dtype]


@pytest.mark.parametrize("grid_cap", CAPS, indirect=True)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("ns,m", [(3, 9), (6, 8), (8, 6)])
def test_wide_gates_multitile(ns, m, dtype, grid_cap):
    """Controlled evolutions (vector GEMM, matrix cores, LDS-staged matrix
    cores), UCRY and diagonal sweeps under a bounded grid."""
    n = ns + m + 1
    gates = W.wide_gate_circuit(ns, m, 700 + ns)
    psi0 = W.random_state(n, 700 + ns)
    _say(f"multitile wide gates ns={ns} m={m} dtype={dtype} cap={grid_cap}")
    want = _oracle_apply(("wg", ns, m), psi0, n, gates)
    for k in (None, 4):
        got, fams = _run(n, gates, psi0, dtype, k)
        _say(f"  k={k} families {sorted(fams)}")
        assert np.max(np.abs(got - want)) <= TOL[dtype], k


@pytest.mark.parametrize("grid_cap", CAPS, indirect=True)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k,control", [(4, True), (6, False), (7, True), (8, True)])
def test_matrix_core_wide_multitile(k, control, dtype, grid_cap):
    """Wide gates of 16..64 columns on >= 16384 rows (matrix cores) and 128
    or 256 columns on >= 2048 rows (rows staged in LDS), bounded grid."""
    n = k + (15 if k <= 6 else 12) + (1 if control else 0)
    rng = np.random.default_rng(800 + k + (100 if control else 0))
    qs = rng.choice(n, size=k + (1 if control else 0), replace=False).tolist()
    U = W.random_unitary(1 << k, rng)
    g = W.Gate("cdense" if control else "dense", tuple(qs), np.ascontiguousarray(U).view(np.float64).ravel())
    _say(f"multitile matrix-core wide n={n} qubits={qs} dtype={dtype} cap={grid_cap}")
    psi0 = W.random_state(n, 9 * k)
    want = _oracle_apply(("mc", k, control), psi0, n, [g])
    got, fams = _run(n, [g], psi0, dtype)
    assert fams == {"wide"}
    assert np.max(np.abs(got - want)) <= TOL[dtype]


@pytest.mark.parametrize("grid_cap", [1, 8], indirect=True)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_hhl_64bus_multitile(dtype, grid_cap):
    """The 64-bus, 10-clock-qubit HHL solve, fused at k = 4, with every launch
    bounded: full state and x_hat against the oracle."""
    hs = _hs()
    A, b = W.dc_powerflow(64, 0)
    if "hhl64" not in _ORACLE:
        _ORACLE["hhl64"] = oracle.hhl_solve(A, b, 10)
    psi_ref, _, xh_ref, _ = _ORACLE["hhl64"]
    c = hs.circuit_build_hhl(A, b, 10)
    s = hs.sv_create(c.n_qubits, dtype)
    s.apply_timed(hs.fuse(c, 4))
    err = float(np.max(np.abs(s.get() - psi_ref)))
    x_hat, _ = s.postselect_solution(c, 63)
    s.close()
    _say(f"multitile 64-bus {dtype} cap={grid_cap}: max|d amp|={err:.3e}")
    assert err <= TOL[dtype]
    assert float(np.dot(x_hat, xh_ref) ** 2) >= 0.999
