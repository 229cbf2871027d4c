"""GPU test of sv_postselect_solution_noalloc, the readout entry point that
allocates nothing: on caller-owned device memory (here a state's buffer,
handed out by sv_device_buffer) it must return what sv_postselect_solution
returns, call after call (the second call on a smaller state), at the
parity bar of each precision."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

# parity bar of each precision (max |difference|)
TOL = {"c128": 1e-12, "c64": 2e-5}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noalloc_readout_matches_existing_entry_point(dtype):
    import paper_2402_08136_amd as hs

    # first a 16-bus system (4 system + 6 clock qubits), then a smaller
    # 4-bus one (2 + 4): the shared scratch keeps the first call's contents
    for nbus, m, seed in ((16, 6, 11), (4, 4, 12)):
        A, b = W.dc_powerflow(nbus, seed)
        c = hs.circuit_build_hhl(A, b, m)
        n = c.n_qubits
        _say(f"[noalloc] {dtype} {nbus}-bus m={m} n={n}")
        s = hs.sv_create(n, dtype)
        s.apply(hs.fuse(c, 3))
        x_ref, info_ref = s.postselect_solution(c, b.size)
        ptr, nbytes, stream = s.device_buffer()
        assert nbytes == (16 if dtype == "c128" else 8) << n
        x_na, info_na = hs.sv_postselect_solution_noalloc(ptr, nbytes, n, dtype, stream, c, b.size)
        assert np.max(np.abs(x_na - x_ref)) <= TOL[dtype]
        for key in ("scale", "p_anc1", "p_anc1_clock0", "max_imag", "pad_leak"):
            assert abs(info_na[key] - info_ref[key]) <= TOL[dtype], key
        s.close()


def test_noalloc_rejects_oversized_block():
    """More than 10 system qubits is beyond the fixed scratch: a clear error
    before any device work."""
    import paper_2402_08136_amd as hs

    A = np.eye(1025) * 2.0
    b = np.ones(1025)
    c = hs.circuit_build_hhl(A, b, 2, device_evolutions=True)
    s = hs.sv_create(c.n_qubits, "c128")
    ptr, nbytes, stream = s.device_buffer()
    with pytest.raises(hs.HHLSVError) as ei:
        hs.sv_postselect_solution_noalloc(ptr, nbytes, c.n_qubits, "c128", stream, c, 1025)
    assert "10 system qubits" in str(ei.value)
    s.close()
