"""Mirror circuits on the full 33-qubit state.

A circuit C followed by its inverse C-dagger returns |0...0> exactly, so on
the 33-qubit state (128 GiB at complex128, 64 GiB at complex64), which the
oracle cannot hold, amplitude 0 must come back to 1 and every other amplitude
to 0.  C is four layers of the throughput workload (H, RZ and U3 on every
qubit, CX on a random matching, seed 2402); C and C-dagger are fused as two
separate circuits, so every sweep kernel runs in its full-size launch shape:
each wave walks many tiles through its XCD slice.  A wrong tile stride or
slice bound leaves some amplitudes unvisited or visited twice, which breaks
the identity even where it keeps the norm.

Bars: |amp_0 - 1| <= 1e-10 (complex128), <= 2e-5 (complex64), and the same
bar on max |amp| over sampled other indices.
"""
import sys

import numpy as np
import pytest

import workloads as W
from _ref import inverse_gates

pytestmark = pytest.mark.gpu

N = 33
TOL = {"c128": 1e-10, "c64": 2e-5}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [4, 5])
def test_mirror_33q(k, dtype):
    import paper_2402_08136_amd as hs
    gates = W.layered_circuit(N, 4, 2402)
    fwd = hs.fuse(hs.circuit_from_gates(N, gates), k)
    inv = hs.fuse(hs.circuit_from_gates(N, inverse_gates(gates)), k)
    _say(f"mirror n={N} k={k} dtype={dtype}: {fwd.n_gates} + {inv.n_gates} sweeps")
    s = hs.sv_create(N, dtype)
    try:
        ms_f, fam_f = s.apply_timed(fwd)
        # after C alone the state is spread out: amplitude 0 is far from 1
        a0_mid = complex(s.get(0, 1)[0])
        ms_i, fam_i = s.apply_timed(inv)
        a0 = complex(s.get(0, 1)[0])
        rng = np.random.default_rng(33 + k)
        idx = np.unique(np.concatenate([
            rng.integers(1, 1 << N, size=4096, dtype=np.int64),
            np.arange(1, 4096, dtype=np.int64),                 # low block
            (1 << N) - 1 - np.arange(4096, dtype=np.int64),     # top block
            (np.int64(1) << np.arange(N, dtype=np.int64))[1:],  # one-hot
        ]))
        rest = s.get_at(idx)
        norm2 = s.norm2()
    finally:
        s.close()
    fams = sorted({hs.KERNEL_FAMILY[int(f)] for f in np.concatenate([fam_f, fam_i])})
    rate = 2 * (1 << N) * (16 if dtype == "c128" else 8) / (np.median(np.concatenate([ms_f, ms_i])) * 1e-3)
    _say(f"  |amp0 - 1| = {abs(a0 - 1):.3e} (after C: |amp0| = {abs(a0_mid):.3e}); "
         f"max |other| = {np.max(np.abs(rest)):.3e}; |norm2 - 1| = {abs(norm2 - 1):.3e}; "
         f"median sweep {rate / 1e9:.0f} GB/s; families {fams}")
    assert abs(a0_mid) < 0.5
    assert abs(a0 - 1) <= TOL[dtype]
    assert np.max(np.abs(rest)) <= TOL[dtype]
    assert abs(norm2 - 1) <= 10 * TOL[dtype]
