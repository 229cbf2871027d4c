"""GPU parity of the signed (sign-qubit) and dilated HHL paths: the HIP path
through the C-ABI against the CPU oracle run with the same variant, on the
same seeded inputs.  Single state (full state compared element by element),
batched persistent kernel and the serving loop.

Bars: complex128 max |delta amplitude| <= 1e-12, complex64 <= 2e-5; x_hat
compared with the oracle's scaled by ||Re y|| (an amplitude error e moves
x_hat by about e / ||Re y||).
"""
import sys
import time

import numpy as np
import pytest

import oracle
import workloads as W
from _ref import AMP_TOL, check_postselected, oracle_postselected

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 2e-5}
OFLAGS = {"signed": oracle.HHL_SIGNED, "dilate": oracle.HHL_DILATE, "gauss_seidel": oracle.HHL_GS}


def _hs():
    import paper_2402_08136_amd as hs
    return hs


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cases():
    """(label, mode, A, b, m, t): indefinite, negative definite, exact and
    off-grid non-symmetric, the 29 x 29 dilated shape (6 data qubits), and
    Gauss-Seidel preconditioned power-flow systems (14- and 30-bus shapes)."""
    out = []
    A, b, t, _ = W.signed_spectrum_system(3, 7, 21)
    out.append(("signed-exact", "signed", A, b, 7, t))
    A, b = W.general_system(13, 22, kappa=60.0, symmetric=True)
    out.append(("signed-13", "signed", A, b, 8, 0.0))
    A, b = W.dc_powerflow(16, 23)
    out.append(("negdef-16", "signed", -A, b, 8, 0.0))
    A, b, t, _ = W.nonsymmetric_exact_system(6, 7, 24)
    out.append(("dilate-exact", "dilate", A, b, 7, t))
    A, b = W.general_system(5, 25, kappa=20.0)
    out.append(("dilate-5", "dilate", A, b, 7, 0.0))
    A, b = W.general_system(29, 26, kappa=100.0)
    out.append(("dilate-29", "dilate", A, b, 8, 0.0))
    A, b = W.dc_powerflow(14, 27)
    out.append(("gs-14bus", "gauss_seidel", A, b, 7, 0.0))
    A, b = W.dc_powerflow(30, 0)
    out.append(("gs-30bus", "gauss_seidel", A, b, 8, 0.0))
    return out


CASES = _cases()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [None, 2, 4])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_signed_dilated_state_parity(case, k, dtype):
    hs = _hs()
    label, mode, A, b, m, t = CASES[case]
    _say(f"signed/dilated parity {label} k={k} {dtype}")
    psi_ref, x_ref, xh_ref, info_ref = oracle.hhl_solve(A, b, m, t, flags=OFLAGS[mode])
    c = hs.circuit_build_hhl(A, b, m, t, mode=mode, device_evolutions=(k == 4))
    run = hs.fuse(c, k) if k else c
    s = hs.sv_create(c.n_qubits, dtype)
    s.apply(run)
    psi = s.get()
    x_hat, info = s.postselect_solution(c, b.size)
    s.close()
    err = float(np.max(np.abs(psi - psi_ref)))
    _say(f"  n={c.n_qubits} max|d amp|={err:.3e}")
    assert err <= TOL[dtype]
    scale = np.sqrt(max(info_ref["p10"], 1e-30))
    assert np.max(np.abs(x_hat - xh_ref)) * scale <= 2 * TOL[dtype]
    assert abs(info["p_anc1"] - info_ref["p1"]) <= 2 * TOL[dtype]
    assert abs(info["p_anc1_clock0"] - info_ref["p10"]) <= 2 * TOL[dtype]
    assert abs(info["pad_leak"] - info_ref["pad_leak"]) <= 2 * TOL[dtype] + 1e-14
    if dtype == "c128":
        x = info["scale"] * x_hat
        assert np.linalg.norm(x - x_ref) <= 1e-10 * np.linalg.norm(x_ref)
        if label.endswith("exact"):
            xs = np.linalg.solve(A, b)
            assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_signed_dilated_batch_matches_oracle(dtype):
    """SPD, signed and dilated instances side by side in one batched launch."""
    hs = _hs()
    items = []
    A, b = W.dc_powerflow(4, 30)
    items.append(("spd", A, b, 5, 0.0))
    for label, mode, A, b, m, t in CASES:
        if A.shape[0] <= 13:
            items.append((mode, A, b, m, t))
    A, b = W.general_system(3, 31, kappa=8.0)
    items.append(("dilate", A, b, 5, 0.0))
    A, b = W.general_system(4, 32, kappa=8.0, symmetric=True)
    items.append(("signed", A, b, 6, 0.0))
    A, b = W.dc_powerflow(8, 33)
    items.append(("gauss_seidel", A, b, 6, 0.0))
    bt = hs.Batch(dtype, 3)
    circs = []
    for mode, A, b, m, t in items:
        c = hs.circuit_build_hhl(A, b, m, t, mode=mode, device_evolutions=True)
        circs.append(c)
        bt.add(c)
    ms = bt.run()
    _say(f"signed/dilated batch {dtype}: {len(bt)} instances in {ms:.3f} ms")
    tol = AMP_TOL[dtype]
    for i, (mode, A, b, m, t) in enumerate(items):
        ref = oracle_postselected(A, b, m, OFLAGS.get(mode, 0), t)
        info_ref = ref[1]
        x_hat, info = bt.solution(i)
        y, p1 = bt.postselected(i)
        check_postselected(y, p1, x_hat, ref, dtype, (i, mode))
        assert abs(info["p_anc1_clock0"] - info_ref["p10"]) <= 2 * tol * np.sqrt(y.size)
        assert abs(info["pad_leak"] - info_ref["pad_leak"]) <= 2 * tol * np.sqrt(y.size)


def _wait_all(srv, tickets, timeout=120.0, y_counts=None):
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        for t in tickets:
            if t not in res:
                r = srv.poll_ex(t, y_counts[t]) if y_counts else srv.poll(t)
                if r is not None:
                    res[t] = r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(tickets) - len(res)} requests still pending")
        time.sleep(0.002)
    return res


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("lds", [0, -1])
def test_serving_auto_mode_matches_oracle(dtype, lds):
    """A server in auto mode: SPD, indefinite and non-symmetric requests
    each get the variant the builder picks, and match the oracle's run of it."""
    hs = _hs()
    reqs = []
    for i in range(4):
        A, b = W.dc_powerflow(4 + 4 * i, 40 + i)
        reqs.append((0, A, b, 6))
        S, bs = W.general_system(3 + 2 * i, 50 + i, kappa=10.0, symmetric=True)
        reqs.append((oracle.HHL_SIGNED, S, bs, 7))
        G, bg = W.general_system(3 + 3 * i, 60 + i, kappa=10.0)
        reqs.append((oracle.HHL_DILATE, G, bg, 7))
    srv = hs.Server(dtype, k_max=3, mode="auto", lds_max_qubits=lds)
    tickets = [srv.submit(A, b, m) for _, A, b, m in reqs]
    refs = {t: oracle_postselected(A, b, m, fl) for t, (fl, A, b, m) in zip(tickets, reqs)}
    res = _wait_all(srv, tickets, y_counts={t: 1 << refs[t][1]["ns"] for t in tickets})
    for t in tickets:
        x_hat, info, y, p1 = res[t]
        check_postselected(y, p1, x_hat, refs[t], dtype, t)
    st = srv.stats()
    _say(f"serve auto {dtype}: {st}")
    assert st["done"] == len(reqs) and st["failed"] == 0
    srv.stop()
