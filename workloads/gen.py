"""Seeded generators for every workload shape used by tests and the benchmark.

All draws go through ``random.Random(seed)`` (MT19937, identical on every
platform) or ``numpy.random.default_rng(seed)``.  Nothing here implements the
HHL method: the generators return plain arrays and gate lists which the CPU
oracle and the device library each consume with their own code.

Gate lists are lists of ``Gate(kind, qubits, params)`` with ``kind`` one of
the strings below and ``params`` a float64 numpy array:

  'h', 'x'                 qubits (q,)             params []
  'ry', 'rz', 'p'          qubits (q,)             params [angle]
  'u3'                     qubits (q,)             params [theta, phi, lam]
  'cx'                     qubits (control, target)
  'cp'                     qubits (a, b)           params [phi]
  'swap'                   qubits (a, b)
  'dense'                  qubits (q0..q_{k-1})    params: 2^k x 2^k complex
                                                   matrix, row-major,
                                                   interleaved (re, im); the
                                                   matrix index is
                                                   sum_l bit(q_l) * 2^l
  'cdense'                 qubits (c, q0..q_{k-1}) as 'dense', applied where
                                                   bit c is 1
  'ucry'                   qubits (t, c0..c_{r-1}) params: 2^r angles; RY of
                                                   angle[sum_l bit(c_l) 2^l]
                                                   acts on qubit t
"""
from __future__ import annotations

import math
import random
from collections import namedtuple

import numpy as np

__all__ = [
    "Gate", "dc_powerflow", "layered_circuit", "random_unitary",
    "random_state", "random_circuit", "wide_gate_circuit", "batch_specs",
    "serve_specs", "exact_spectrum_system", "split_register_circuit",
    "flatten_circuit", "TWO_PI", "signed_spectrum_system",
    "nonsymmetric_exact_system", "general_system", "ac_powerflow_case",
]

TWO_PI = 2.0 * math.pi

Gate = namedtuple("Gate", "kind qubits params")


def _g(kind, qubits, params=()):
    return Gate(kind, tuple(int(q) for q in qubits),
                np.asarray(params, dtype=np.float64).ravel())


# --------------------------------------------------------------------------
# DC power-flow systems (stand-in for the IEEE cases the paper draws from
# MATPOWER, Sec. IV): B' of a random connected graph with the slack bus
# removed, and injections P.
# --------------------------------------------------------------------------
def dc_powerflow(n_bus: int, seed: int, extra_frac: float = 0.3,
                 b_lo: float = 5.0, b_hi: float = 20.0):
    """Reduced DC power-flow system for a random connected ``n_bus`` graph.

    Graph: a random spanning tree (a Fisher-Yates permutation ``perm``; bus
    ``perm[i]`` attaches to ``perm[j]`` with ``j`` uniform in ``[0, i)``) plus
    ``round(extra_frac * (n_bus - 1))`` extra edges drawn from the non-edges.
    Line susceptances ~ U[b_lo, b_hi].  The susceptance Laplacian with the
    slack bus 0 removed is ``A`` ((n_bus-1) x (n_bus-1), symmetric positive
    definite); ``b`` holds injections ~ N(0, 1) at buses 1..n_bus-1.
    """
    if n_bus < 2:
        raise ValueError("need at least 2 buses")
    rng = random.Random(seed)
    perm = list(range(n_bus))
    rng.shuffle(perm)
    edges = set()
    for i in range(1, n_bus):
        j = rng.randrange(i)
        a, b = perm[i], perm[j]
        edges.add((min(a, b), max(a, b)))
    n_extra = int(round(extra_frac * (n_bus - 1)))
    non_edges = [(a, b) for a in range(n_bus) for b in range(a + 1, n_bus)
                 if (a, b) not in edges]
    n_extra = min(n_extra, len(non_edges))
    for e in rng.sample(non_edges, n_extra):
        edges.add(e)
    lap = np.zeros((n_bus, n_bus))
    for (a, b) in sorted(edges):
        s = rng.uniform(b_lo, b_hi)
        lap[a, a] += s
        lap[b, b] += s
        lap[a, b] -= s
        lap[b, a] -= s
    A = np.ascontiguousarray(lap[1:, 1:])
    bvec = np.array([rng.gauss(0.0, 1.0) for _ in range(n_bus - 1)])
    return A, bvec


def exact_spectrum_system(ns: int, m: int, seed: int, k_lo: int | None = None,
                          delta: float = 0.25):
    """SPD system whose eigenvalues are ``delta * k_i`` with integer ``k_i``.

    With ``t = 2*pi / (2^m * delta)`` every eigenvalue maps to an integer
    clock value, so phase estimation is exact (the textbook HHL identity of
    Sec. III-A applies without discretisation error).  Returns
    ``(A, b, t, k)`` with ``A = Q diag(delta*k) Q^T`` for a seeded random
    orthogonal ``Q``.
    """
    rng = np.random.default_rng(seed)
    dim = 1 << ns
    top = (1 << m) - 1
    if k_lo is None:
        k_lo = max(1, top // 8)
    k = rng.integers(k_lo, top + 1, size=dim)
    k[0] = k_lo                      # the smallest eigenvalue is present
    z = rng.standard_normal((dim, dim))
    q, r = np.linalg.qr(z)
    q = q * np.sign(np.diag(r))
    A = (q * (delta * k)) @ q.T
    A = 0.5 * (A + A.T)
    b = rng.standard_normal(dim)
    t = TWO_PI / ((1 << m) * delta)
    return A, b, t, k


def ac_powerflow_case(n_bus: int, seed: int, extra_frac: float = 0.3,
                      pv_frac: float = 0.2):
    """Seeded synthetic AC power-flow case (stands in for the IEEE cases).

    Network: a random spanning tree plus ``round(extra_frac * (n_bus - 1))``
    extra branches, as in ``dc_powerflow``.  Branch reactance x ~ U[0.05,
    0.25] p.u., resistance r = x * U[0.1, 0.3], total line charging
    b ~ U[0, 0.04].  Bus 0 is the slack (|V| = 1.02); about ``pv_frac`` of
    the others are PV buses (|V| ~ U[0.99, 1.04], generation ~ U[0.1, 0.4]);
    every non-slack bus carries a load P ~ U[0.02, 0.12], Q ~ U[0.01, 0.05].
    Returns a dict of arrays: from, to, r, x, bsh, type (0 slack, 1 PV,
    2 PQ), p, q (net injections), vset.
    """
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n_bus)
    edges = set()
    for i in range(1, n_bus):
        j = int(rng.integers(0, i))
        a, b = int(perm[i]), int(perm[j])
        edges.add((min(a, b), max(a, b)))
    n_extra = int(round(extra_frac * (n_bus - 1)))
    tries = 0
    while n_extra > 0 and tries < 100 * n_bus:
        tries += 1
        a, b = (int(v) for v in rng.integers(0, n_bus, size=2))
        if a == b or (min(a, b), max(a, b)) in edges:
            continue
        edges.add((min(a, b), max(a, b)))
        n_extra -= 1
    edges = sorted(edges)
    fr = np.array([e[0] for e in edges], dtype=np.int32)
    to = np.array([e[1] for e in edges], dtype=np.int32)
    x = rng.uniform(0.05, 0.25, size=len(edges))
    r = x * rng.uniform(0.1, 0.3, size=len(edges))
    bsh = rng.uniform(0.0, 0.04, size=len(edges))
    typ = np.full(n_bus, 2, dtype=np.int32)
    typ[0] = 0
    vset = np.ones(n_bus)
    vset[0] = 1.02
    pv = rng.uniform(size=n_bus) < pv_frac
    pv[0] = False
    typ[pv] = 1
    vset[pv] = rng.uniform(0.99, 1.04, size=int(pv.sum()))
    p = -rng.uniform(0.02, 0.12, size=n_bus)
    q = -rng.uniform(0.01, 0.05, size=n_bus)
    p[pv] += rng.uniform(0.1, 0.4, size=int(pv.sum()))
    p[0] = q[0] = 0.0
    return {"from": fr, "to": to, "r": r, "x": x, "bsh": bsh, "type": typ,
            "p": p, "q": q, "vset": vset}


def _orthogonal(dim: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed real orthogonal ``dim x dim`` matrix."""
    z = rng.standard_normal((dim, dim))
    q, r = np.linalg.qr(z)
    return q * np.sign(np.diag(r))


def signed_spectrum_system(ns: int, m: int, seed: int, k_lo: int | None = None,
                           delta: float = 0.25):
    """Symmetric indefinite system with eigenvalues ``+-delta * k_i``.

    ``k_i`` are integers in ``[k_lo, 2^(m-1) - 1]`` with seeded signs (both
    signs present when the dimension allows), so with
    ``t = 2*pi / (2^m * delta)`` every eigenvalue maps to an integer clock
    value that fits an m-bit two's-complement register.  Returns
    ``(A, b, t, signed_k)``.
    """
    rng = np.random.default_rng(seed)
    dim = 1 << ns
    top = (1 << (m - 1)) - 1
    if k_lo is None:
        k_lo = max(1, top // 8)
    k = rng.integers(k_lo, top + 1, size=dim)
    k[0] = k_lo
    sg = rng.choice([-1, 1], size=dim)
    if dim > 1:
        sg[0], sg[1] = -1, 1
    else:
        sg[0] = -1
    q = _orthogonal(dim, rng)
    lam = delta * sg * k
    A = (q * lam) @ q.T
    A = 0.5 * (A + A.T)
    b = rng.standard_normal(dim)
    t = TWO_PI / ((1 << m) * delta)
    return A, b, t, sg * k


def nonsymmetric_exact_system(N: int, m: int, seed: int,
                              k_lo: int | None = None, delta: float = 0.25):
    """Non-symmetric ``N x N`` system ``A = U diag(delta * k) W^T``.

    ``U`` and ``W`` are independent seeded random orthogonal matrices and
    ``k_i`` integers in ``[k_lo, 2^(m-1) - 1]``, so the singular values, and
    with them the +- eigenvalues of the dilated system, sit on the clock grid
    of ``t = 2*pi / (2^m * delta)``.  Returns ``(A, b, t, k)``.
    """
    rng = np.random.default_rng(seed)
    top = (1 << (m - 1)) - 1
    if k_lo is None:
        k_lo = max(1, top // 8)
    k = rng.integers(k_lo, top + 1, size=N)
    k[0] = k_lo
    u = _orthogonal(N, rng)
    w = _orthogonal(N, rng)
    A = (u * (delta * k)) @ w.T
    b = rng.standard_normal(N)
    t = TWO_PI / ((1 << m) * delta)
    return A, b, t, k


def general_system(N: int, seed: int, kappa: float = 20.0,
                   symmetric: bool = False, negative_frac: float = 0.5):
    """Seeded well-posed system with condition number ``kappa``.

    ``symmetric=False``: ``A = U diag(s) W^T`` with singular values ``s``
    log-uniform in ``[1, kappa]`` (the extremes present).
    ``symmetric=True``: ``A = Q diag(s * sign) Q^T`` with about
    ``negative_frac`` of the eigenvalues negative.  Returns ``(A, b)``.
    """
    rng = np.random.default_rng(seed)
    s = np.exp(rng.uniform(0.0, math.log(kappa), size=N))
    s[0] = 1.0
    if N > 1:
        s[-1] = kappa
    if symmetric:
        sg = np.where(rng.uniform(size=N) < negative_frac, -1.0, 1.0)
        q = _orthogonal(N, rng)
        A = (q * (s * sg)) @ q.T
        A = 0.5 * (A + A.T)
    else:
        A = (_orthogonal(N, rng) * s) @ _orthogonal(N, rng).T
    b = rng.standard_normal(N)
    return A, b


# --------------------------------------------------------------------------
# Random circuits
# --------------------------------------------------------------------------
def random_unitary(dim: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed ``dim x dim`` unitary (QR of a complex Gaussian)."""
    z = (rng.standard_normal((dim, dim)) +
         1j * rng.standard_normal((dim, dim))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))


def _cplx_params(mat: np.ndarray) -> np.ndarray:
    mat = np.ascontiguousarray(mat, dtype=np.complex128)
    return mat.view(np.float64).ravel().copy()


def random_state(n: int, seed: int) -> np.ndarray:
    """Normalised complex Gaussian state of ``n`` qubits (complex128)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def layered_circuit(n: int, layers: int, seed: int):
    """Random layered circuit of the 33-qubit throughput workload.

    Each layer applies H, RZ(theta ~ U[0, 2pi)) and U3(theta, phi, lambda,
    each ~ U[0, 2pi)) on every qubit, then CX on a random matching: a random
    permutation of the qubits paired off in order (control first).  For odd
    ``n`` one qubit per layer stays idle.
    """
    rng = random.Random(seed)
    gates = []
    for _ in range(layers):
        for q in range(n):
            gates.append(_g("h", (q,)))
            gates.append(_g("rz", (q,), [rng.uniform(0.0, TWO_PI)]))
            gates.append(_g("u3", (q,), [rng.uniform(0.0, TWO_PI)
                                        for _ in range(3)]))
        perm = list(range(n))
        rng.shuffle(perm)
        for i in range(n // 2):
            gates.append(_g("cx", (perm[2 * i], perm[2 * i + 1])))
    return gates


def split_register_circuit(n: int, layers: int, seed: int):
    """Layered circuit on two interleaved, non-interacting registers.

    Register 0 holds the even qubits, register 1 the odd ones; CX pairs never
    cross registers, so the output state of ``|0...0>`` is the tensor product
    of the two register states.  Returns ``(gates, regs)`` where ``regs[r]``
    lists the global qubits of register ``r`` (its local qubit ``i`` is
    ``regs[r][i]``).
    """
    rng = random.Random(seed)
    regs = [list(range(0, n, 2)), list(range(1, n, 2))]
    gates = []
    for _ in range(layers):
        for q in range(n):
            gates.append(_g("h", (q,)))
            gates.append(_g("rz", (q,), [rng.uniform(0.0, TWO_PI)]))
            gates.append(_g("u3", (q,), [rng.uniform(0.0, TWO_PI)
                                        for _ in range(3)]))
        for reg in regs:
            perm = list(reg)
            rng.shuffle(perm)
            for i in range(len(perm) // 2):
                gates.append(_g("cx", (perm[2 * i], perm[2 * i + 1])))
    return gates, regs


_ONE_Q = ("h", "x", "ry", "rz", "p", "u3")
_TWO_Q = ("cx", "cp", "swap")


def random_circuit(n: int, n_gates: int, seed: int, kmax: int = 5,
                   kinds=None, qubit_pool=None):
    """Random mix of every gate kind on random qubits of an ``n``-qubit state.

    ``kinds`` restricts the kinds drawn; ``qubit_pool`` restricts the qubits
    (e.g. to force low or high targets).  Dense and controlled-dense gates
    carry Haar-random unitaries of up to ``kmax`` qubits; UCRY gates carry
    angles ~ U[0, 2pi).
    """
    rng = random.Random(seed)
    nrng = np.random.default_rng(seed + 7919)
    pool = list(range(n)) if qubit_pool is None else list(qubit_pool)
    if kinds is None:
        kinds = list(_ONE_Q + _TWO_Q) + ["dense", "cdense", "ucry"]
    gates = []
    for _ in range(n_gates):
        kind = rng.choice(kinds)
        if kind in _ONE_Q:
            q = rng.choice(pool)
            npar = {"h": 0, "x": 0, "ry": 1, "rz": 1, "p": 1, "u3": 3}[kind]
            gates.append(_g(kind, (q,), [rng.uniform(0, TWO_PI)
                                         for _ in range(npar)]))
        elif kind in _TWO_Q:
            if len(pool) < 2:
                continue
            a, b = rng.sample(pool, 2)
            gates.append(_g(kind, (a, b),
                            [rng.uniform(0, TWO_PI)] if kind == "cp" else []))
        elif kind == "dense":
            k = rng.randint(1, min(kmax, len(pool)))
            qs = rng.sample(pool, k)
            gates.append(_g("dense", qs,
                            _cplx_params(random_unitary(1 << k, nrng))))
        elif kind == "cdense":
            if len(pool) < 2:
                continue
            k = rng.randint(1, min(kmax, len(pool) - 1))
            qs = rng.sample(pool, k + 1)
            gates.append(_g("cdense", qs,
                            _cplx_params(random_unitary(1 << k, nrng))))
        elif kind == "ucry":
            r = rng.randint(0, min(4, len(pool) - 1))
            qs = rng.sample(pool, r + 1)
            gates.append(_g("ucry", qs, [rng.uniform(0, TWO_PI)
                                         for _ in range(1 << r)]))
        else:
            raise ValueError(kind)
    return gates


def wide_gate_circuit(ns: int, m: int, seed: int, n_rounds: int = 2):
    """Circuit with the register layout and wide gates of an HHL circuit.

    Qubits: system ``0..ns-1``, clock ``ns..ns+m-1``, ancilla ``ns+m``.  It
    uses Haar-random unitaries on the whole system register controlled by
    each clock qubit, random one- and two-qubit gates on the clock register,
    and a UCRY on the ancilla controlled by the whole clock register with
    random angles.  The gate kinds and widths match the HHL circuit; the
    values are random, so it exercises the same kernels at any tolerance.
    """
    rng = random.Random(seed)
    nrng = np.random.default_rng(seed + 104729)
    n = ns + m + 1
    clock = list(range(ns, ns + m))
    gates = []
    for q in range(ns):
        gates.append(_g("u3", (q,), [rng.uniform(0, TWO_PI) for _ in range(3)]))
    for _ in range(n_rounds):
        for c in clock:
            gates.append(_g("h", (c,)))
        for c in clock:
            gates.append(_g("cdense", [c] + list(range(ns)),
                            _cplx_params(random_unitary(1 << ns, nrng))))
        for _ in range(m):
            a, b = rng.sample(clock, 2) if m >= 2 else (clock[0], clock[0])
            if a != b:
                gates.append(_g("cp", (a, b), [rng.uniform(0, TWO_PI)]))
            gates.append(_g("h", (rng.choice(clock),)))
        if m >= 2:
            a, b = rng.sample(clock, 2)
            gates.append(_g("swap", (a, b)))
        gates.append(_g("ucry", [n - 1] + clock,
                        [rng.uniform(0, TWO_PI) for _ in range(1 << m)]))
    return gates


def flatten_circuit(gates):
    """Flat arrays (kinds, qubit offsets, qubits, param offsets, params)."""
    kinds = [g.kind for g in gates]
    qoff = np.zeros(len(gates) + 1, dtype=np.int32)
    poff = np.zeros(len(gates) + 1, dtype=np.int64)
    for i, g in enumerate(gates):
        qoff[i + 1] = qoff[i] + len(g.qubits)
        poff[i + 1] = poff[i] + len(g.params)
    qubits = np.array([q for g in gates for q in g.qubits], dtype=np.int32)
    params = (np.concatenate([g.params for g in gates]) if gates
              else np.zeros(0)).astype(np.float64)
    return kinds, qoff, qubits, poff, params


# --------------------------------------------------------------------------
# Batch and serving schedules
# --------------------------------------------------------------------------
def batch_specs(count: int = 8192, seed: int = 8136, ns_range=(2, 6),
                m_range=(4, 10)):
    """Per-instance (ns, m, graph_seed) of the batched-solve workload."""
    rng = random.Random(seed)
    out = []
    for _ in range(count):
        ns = rng.randint(*ns_range)
        m = rng.randint(*m_range)
        out.append((ns, m, rng.getrandbits(31)))
    return out


def serve_specs(rate: float = 2000.0, duration: float = 60.0,
                arrival_seed: int = 2000, size_seed: int = 2001,
                ns_range=(3, 8), m_range=(6, 12)):
    """Open-loop Poisson arrivals: list of (arrival_s, ns, m, graph_seed)."""
    arng = random.Random(arrival_seed)
    srng = random.Random(size_seed)
    out = []
    t = 0.0
    while True:
        t += arng.expovariate(rate)
        if t >= duration:
            break
        ns = srng.randint(*ns_range)
        m = srng.randint(*m_range)
        out.append((t, ns, m, srng.getrandbits(31)))
    return out
