"""GPU parity of the Newton-Raphson AC power flow with HHL inner solves: the
library (Jacobian in complex form, HHL circuits run on the GPU) against the
oracle (polar form, HHL simulated gate by gate on the CPU) on the same seeded
synthetic cases, iteration by iteration.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def _hs():
    import paper_2402_08136_amd as hs
    return hs


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("nb,seed,m,mode", [(5, 0, 8, "dilate"), (5, 1, 9, "gauss_seidel"),
                                            (14, 0, 9, "dilate"), (14, 1, 9, "gauss_seidel")])
def test_pf_newton_hhl_matches_oracle(nb, seed, m, mode):
    hs = _hs()
    case = W.ac_powerflow_case(nb, seed)
    flags = oracle.HHL_DILATE if mode == "dilate" else oracle.HHL_GS
    vo, ao, io = oracle.pf_newton(case, "hhl", m=m, flags=flags, max_iter=25, tol=1e-8)
    for dtype, k in (("c128", None), ("c128", 3), ("c64", 3)):
        vm, va, info = hs.pf_newton(case, m, mode=mode, dtype=dtype, k_max=k or 0, max_iter=25, tol=1e-8)
        _say(f"pf {nb}-bus seed={seed} m={m} {mode} {dtype} k={k}: it={info['iterations']} "
             f"(oracle {io['iterations']}) mismatch={info['mismatch']:.2e} hhl {info['hhl_seconds']:.3f}s")
        assert info["converged"] and io["converged"]
        if dtype == "c128":
            # each inner solve agrees to ~1e-12, so the iterates do too
            assert info["iterations"] == io["iterations"]
            hist, ref = np.array(info["history"]), np.array(io["history"])
            assert np.all(np.abs(hist - ref) <= 1e-9 * np.maximum(ref, 1e-6) + 1e-12)
            assert np.abs(vm - vo).max() < 1e-9 and np.abs(va - ao).max() < 1e-9
        else:
            # FP32 states perturb each step by ~1e-5 relative; Newton still
            # reaches the same operating point
            assert np.abs(vm - vo).max() < 1e-6 and np.abs(va - ao).max() < 1e-6


def test_pf_newton_hhl_reaches_exact_operating_point():
    """30-bus case, 9 clock qubits, device-built evolutions: HHL-Newton lands
    on the operating point exact Newton finds."""
    hs = _hs()
    case = W.ac_powerflow_case(30, 3)
    v0, a0, _ = oracle.pf_newton(case, "ge")
    vm, va, info = hs.pf_newton(case, 9, mode="dilate", k_max=3, max_iter=40, tol=1e-9,
                                device_evolutions=True)
    _say(f"pf 30-bus: {info['iterations']} iterations, {info['n_unknowns']} unknowns, "
         f"hhl {info['hhl_seconds']:.3f}s, history {['%.1e' % h for h in info['history']]}")
    assert info["converged"]
    assert np.abs(vm - v0).max() < 1e-8 and np.abs(va - a0).max() < 1e-8
