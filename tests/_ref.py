"""Small numpy helpers used by the tests to check the oracle and the library
from the outside: tensor-contraction application of a matrix to a state,
circuit inversion, and comparison utilities.

They work by a different mechanism from the oracle's index loop (numpy
tensordot over the qubit axes), so an indexing mistake in either shows up.
"""
from __future__ import annotations

import numpy as np

from workloads import Gate


def apply_tensor(psi: np.ndarray, n: int, qubits, M: np.ndarray,
                 control: int | None = None) -> np.ndarray:
    """Apply a 2^k x 2^k matrix (index r = sum_l bit(q_l) 2^l) by contraction.

    The state is viewed as an n-way tensor whose axis ``a`` is qubit
    ``n-1-a`` (C order of the amplitude index).
    """
    qubits = list(qubits)
    k = len(qubits)
    if control is not None:
        idx = np.arange(1 << n)
        mask = ((idx >> control) & 1).astype(bool)
        on = np.where(mask, psi, 0)
        return np.where(mask, apply_tensor(on, n, qubits, M), psi)
    T = np.asarray(psi, dtype=np.complex128).reshape((2,) * n)
    Mt = np.asarray(M, dtype=np.complex128).reshape((2,) * (2 * k))
    axes_in = [n - 1 - q for q in reversed(qubits)]
    res = np.tensordot(Mt, T, axes=(list(range(k, 2 * k)), axes_in))
    res = np.moveaxis(res, list(range(k)), axes_in)
    return res.reshape(-1)


def ry(theta: float) -> np.ndarray:
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def apply_ucry_tensor(psi, n, target, controls, angles):
    idx = np.arange(1 << n)
    val = np.zeros(1 << n, dtype=np.int64)
    for l, c in enumerate(controls):
        val |= ((idx >> c) & 1) << l
    out = np.zeros_like(psi, dtype=np.complex128)
    for v, th in enumerate(angles):
        mask = val == v
        out += np.where(mask, apply_tensor(np.where(mask, psi, 0), n,
                                           [target], ry(th)), 0)
    return out


def cmat(params: np.ndarray, k: int) -> np.ndarray:
    """Complex matrix from interleaved (re, im) params."""
    d = 1 << k
    return np.asarray(params, dtype=np.float64).view(np.complex128).reshape(d, d)


def inverse_gates(gates):
    """The inverse circuit: reversed order, each gate replaced by its inverse."""
    out = []
    for g in reversed(gates):
        p = g.params
        if g.kind in ("h", "x", "cx", "swap"):
            out.append(g)
        elif g.kind in ("ry", "rz", "p", "cp"):
            out.append(Gate(g.kind, g.qubits, -p))
        elif g.kind == "u3":
            out.append(Gate("u3", g.qubits, np.array([-p[0], -p[2], -p[1]])))
        elif g.kind in ("dense", "cdense"):
            k = len(g.qubits) - (1 if g.kind == "cdense" else 0)
            M = cmat(p, k).conj().T
            out.append(Gate(g.kind, g.qubits,
                            np.ascontiguousarray(M).view(np.float64).ravel()))
        elif g.kind == "ucry":
            out.append(Gate("ucry", g.qubits, -p))
        else:
            raise ValueError(g.kind)
    return out


def oracle_postselected(A, b, m, flags=0, t=0.0):
    """The oracle's solve of (A, b) with m clock qubits: (x_hat, info, y)
    with y_s = psi[2^{n-1} + s], s < 2^ns, the postselected block of Sec.
    III-A step 3."""
    import oracle
    psi, _, xh, info = oracle.hhl_solve(A, b, m, t, flags=flags)
    half = 1 << (info["n"] - 1)
    return xh, info, psi[half:half + (1 << info["ns"])].copy()


AMP_TOL = {"c128": 1e-12, "c64": 2e-5}


def check_postselected(y, p1, x_hat, ref, dtype, what=""):
    """A batched or served result against the oracle: the raw block y and
    P(ancilla = 1) at the amplitude bar; x_hat = Re(y)/||Re y|| (over the
    x entries) through the bound an amplitude error e gives it,
    |d x_hat| ||Re y|| <= e (1 + sqrt(2^ns)).  Returns max |d y|."""
    xh_ref, info_ref, y_ref = ref
    tol = AMP_TOL[dtype]
    err_y = float(np.max(np.abs(np.asarray(y) - y_ref)))
    assert err_y <= tol, (what, err_y)
    assert abs(p1 - info_ref["p1"]) <= tol, what
    xo = int(info_ref["x_off"])
    rn = float(np.linalg.norm(y_ref.real[xo:xo + np.size(xh_ref)]))
    assert np.max(np.abs(np.asarray(x_hat) - xh_ref)) * rn <= tol * (1 + np.sqrt(y_ref.size)), what
    return err_y


def max_abs_diff(a, b) -> float:
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) if np.size(a) else 0.0
