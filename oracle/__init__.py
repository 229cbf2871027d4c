"""ctypes wrapper of the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg.  The library never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

HHL_SIGNED = 1   # two's-complement clock (sign qubit)
HHL_DILATE = 2   # [[0, A'], [A'^T, 0]] for a general square A
HHL_GS = 4       # Gauss-Seidel left preconditioning, then the dilation

KIND = {"h": 0, "x": 1, "ry": 2, "rz": 3, "p": 4, "u3": 5, "cx": 6, "cp": 7,
        "swap": 8, "dense": 9, "cdense": 10, "ucry": 11}


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


class HHLInfo(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int), ("m", ctypes.c_int), ("n", ctypes.c_int),
                ("j0", ctypes.c_int),
                ("beta", ctypes.c_double), ("t", ctypes.c_double),
                ("C", ctypes.c_double), ("lambda_lo", ctypes.c_double),
                ("lambda_hi", ctypes.c_double), ("kappa", ctypes.c_double),
                ("p1", ctypes.c_double), ("p10", ctypes.c_double),
                ("max_imag", ctypes.c_double), ("pad_leak", ctypes.c_double),
                ("x_norm", ctypes.c_double), ("x_off", ctypes.c_int),
                ("sign_qubit", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PFInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int),
                ("n_unknowns", ctypes.c_int), ("mismatch", ctypes.c_double),
                ("history", ctypes.c_double * 64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lp = ctypes.POINTER(ctypes.c_long)
        L.orc_apply_gate.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip,
                                     ctypes.c_int, dp, ctypes.c_long]
        L.orc_apply_circuit.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip,
                                        ip, ip, lp, dp]
        L.orc_gate_matrix.argtypes = [ctypes.c_int, dp, dp]
        L.orc_qft.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.c_int]
        L.orc_jacobi.argtypes = [dp, ctypes.c_int, dp, dp, ip]
        L.orc_ge_solve.argtypes = [dp, dp, ctypes.c_int, dp]
        L.orc_qubit_count.argtypes = [ctypes.c_int, ctypes.c_double,
                                      ctypes.c_int, ip, ip, ip]
        L.orc_hhl_solve.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, dp, dp, dp,
                                    ctypes.POINTER(HHLInfo)]
        L.orc_hhl_params.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, ctypes.POINTER(HHLInfo)]
        L.orc_hhl_solve_ex.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_int, dp, dp,
                                       dp, ctypes.POINTER(HHLInfo)]
        L.orc_hhl_params_ex.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_double, ctypes.c_int,
                                        ctypes.POINTER(HHLInfo)]
        L.orc_hhl_system.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, dp,
                                     dp, ip]
        L.orc_pf_eval.argtypes = [ctypes.c_int, ctypes.c_int, ip, ip, dp, dp, dp,
                                  ip, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_pf_newton.argtypes = [ctypes.c_int, ctypes.c_int, ip, ip, dp, dp,
                                    dp, ip, dp, dp, dp, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, dp, dp,
                                    ctypes.POINTER(PFInfo)]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")
    return rc


def apply_circuit(psi: np.ndarray, n: int, gates) -> np.ndarray:
    """Apply a gate list (``workloads.Gate`` tuples) to a copy of ``psi``."""
    out = np.array(psi, dtype=np.complex128, copy=True)
    if out.size != (1 << n):
        raise ValueError("state size does not match n")
    L = lib()
    for g in gates:
        q = np.asarray(g.qubits, dtype=np.int32)
        p = np.ascontiguousarray(g.params, dtype=np.float64)
        pp = _dp(p) if p.size else ctypes.POINTER(ctypes.c_double)()
        _check(L.orc_apply_gate(_dp(out.view(np.float64)), n, KIND[g.kind],
                                _ip(q), len(q), pp, p.size), g.kind)
    return out


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def gate_matrix(kind: str, params=()) -> np.ndarray:
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).ravel())
    if p.size == 0:
        p = np.zeros(1)
    out = np.zeros(16, dtype=np.complex128)
    k = _check(lib().orc_gate_matrix(KIND[kind], _dp(p),
                                     _dp(out.view(np.float64))), kind)
    d = 1 << k
    return out[:d * d].reshape(d, d).copy()


def qft(psi: np.ndarray, n: int, q0: int, m: int, inverse: bool = False):
    out = np.array(psi, dtype=np.complex128, copy=True)
    _check(lib().orc_qft(_dp(out.view(np.float64)), n, q0, m, int(inverse)),
           "qft")
    return out


def jacobi(A: np.ndarray):
    A = np.ascontiguousarray(A, dtype=np.float64)
    N = A.shape[0]
    V = np.zeros((N, N))
    lam = np.zeros(N)
    sw = np.zeros(1, dtype=np.int32)
    _check(lib().orc_jacobi(_dp(A), N, _dp(V), _dp(lam), _ip(sw)), "jacobi")
    return lam, V, int(sw[0])


def ge_solve(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(b.size)
    _check(lib().orc_ge_solve(_dp(A), _dp(b), b.size, _dp(x)), "ge_solve")
    return x


def qubit_count(dim: int, kappa: float, has_negative: bool):
    a = np.zeros(3, dtype=np.int32)
    _check(lib().orc_qubit_count(dim, kappa, int(has_negative), _ip(a[0:]),
                                 _ip(a[1:]), _ip(a[2:])), "qubit_count")
    return int(a[0]), int(a[1]), int(a[2])


def hhl_params(A, b, m: int, t: float = 0.0, flags: int = 0) -> dict:
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    info = HHLInfo()
    _check(lib().orc_hhl_params_ex(_dp(A), _dp(b), b.size, m, t, flags,
                                   ctypes.byref(info)), "hhl_params")
    return info.as_dict()


def hhl_system(A, b, flags: int = 0):
    """The Hermitian system the circuit encodes: (H, b_hat, x_off)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    L = lib()
    null = ctypes.POINTER(ctypes.c_double)()
    d = _check(L.orc_hhl_system(_dp(A), _dp(b), b.size, flags, null, null,
                                ctypes.POINTER(ctypes.c_int)()), "hhl_system")
    H = np.zeros((d, d))
    bh = np.zeros(d)
    xo = np.zeros(1, dtype=np.int32)
    _check(L.orc_hhl_system(_dp(A), _dp(b), b.size, flags, _dp(H), _dp(bh),
                            _ip(xo)), "hhl_system")
    return H, bh, int(xo[0])


def hhl_solve(A, b, m: int, t: float = 0.0, want_state: bool = True,
              flags: int = 0):
    """Full HHL solve: returns (psi or None, x_hhl, x_hat, info dict)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    N = b.size
    info = HHLInfo()
    pr = hhl_params(A, b, m, t, flags)
    n = pr["n"]
    psi = np.zeros(1 << n, dtype=np.complex128) if want_state else None
    x_hhl = np.zeros(N)
    x_hat = np.zeros(N)
    psi_p = (_dp(psi.view(np.float64)) if want_state
             else ctypes.POINTER(ctypes.c_double)())
    _check(lib().orc_hhl_solve_ex(_dp(A), _dp(b), N, m, t, flags, psi_p,
                                  _dp(x_hhl), _dp(x_hat), ctypes.byref(info)),
           "hhl_solve")
    return psi, x_hhl, x_hat, info.as_dict()


def _pf_arrays(case):
    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    return (i32(case["from"]), i32(case["to"]), f64(case["r"]), f64(case["x"]),
            f64(case["bsh"]), i32(case["type"]), f64(case["p"]), f64(case["q"]),
            f64(case["vset"]))


def pf_eval(case, vm, va):
    """(P, Q, F, J) of the power-flow model at magnitudes vm, angles va."""
    fr, to, r, x, b, ty, p, q, vs = _pf_arrays(case)
    nb, nbr = ty.size, fr.size
    vm = np.ascontiguousarray(vm, dtype=np.float64)
    va = np.ascontiguousarray(va, dtype=np.float64)
    P, Q = np.zeros(nb), np.zeros(nb)
    null = ctypes.POINTER(ctypes.c_double)()
    N = _check(lib().orc_pf_eval(nb, nbr, _ip(fr), _ip(to), _dp(r), _dp(x), _dp(b), _ip(ty),
                                 _dp(p), _dp(q), _dp(vm), _dp(va), _dp(P), _dp(Q), null, null),
               "pf_eval")
    F, J = np.zeros(N), np.zeros((N, N))
    _check(lib().orc_pf_eval(nb, nbr, _ip(fr), _ip(to), _dp(r), _dp(x), _dp(b), _ip(ty),
                             _dp(p), _dp(q), _dp(vm), _dp(va), _dp(P), _dp(Q), _dp(F), _dp(J)),
           "pf_eval")
    return P, Q, F, J


def pf_newton(case, solver="ge", m=10, flags=HHL_DILATE, max_iter=30, tol=1e-10):
    """Newton-Raphson power flow; solver "ge" (exact) or "hhl".
    Returns (vm, va, info dict)."""
    fr, to, r, x, b, ty, p, q, vs = _pf_arrays(case)
    nb = ty.size
    vm, va = np.zeros(nb), np.zeros(nb)
    info = PFInfo()
    _check(lib().orc_pf_newton(nb, fr.size, _ip(fr), _ip(to), _dp(r), _dp(x), _dp(b), _ip(ty),
                               _dp(p), _dp(q), _dp(vs), 0 if solver == "ge" else 1, m, flags,
                               max_iter, tol, _dp(vm), _dp(va), ctypes.byref(info)), "pf_newton")
    d = {"iterations": info.iterations, "converged": bool(info.converged),
         "n_unknowns": info.n_unknowns, "mismatch": info.mismatch,
         "history": list(info.history[:min(info.iterations + 1, 64)])}
    return vm, va, d
