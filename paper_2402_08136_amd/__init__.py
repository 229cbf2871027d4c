"""Python binding of libhhlsv, the MI355X HHL state-vector simulator.

Argument marshalling only: every step runs in the C++/HIP library
(``libhhlsv.so``, built in-tree by ``build.py``).  Importing this module
fails loudly when the library has not been built; there is no fallback.

The functions keep the C-ABI names (``sv_create``, ``circuit_build_hhl``,
``fuse``, ``sv_apply``, ``sv_postselect_solution`` ...) and raise
``HHLSVError`` on a non-OK status.  ``State`` and ``Circuit`` are small
owning wrappers around the handles.  Torch, when used, only supplies device
memory (``State.from_tensor``) and streams (``State.set_stream``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhhlsv.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
        "or `python paper_2402_08136_amd/build.py` (hipcc for gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

C128, C64 = 0, 1
DTYPES = {"c128": C128, "c64": C64, C128: C128, C64: C64}
KIND = {"h": 0, "x": 1, "ry": 2, "rz": 3, "p": 4, "u3": 5, "cx": 6, "cp": 7,
        "swap": 8, "dense": 9, "cdense": 10, "ucry": 11, "diag": 12, "mux2": 13,
        "mux3": 14}
KIND_NAME = {v: k for k, v in KIND.items()}
KERNEL_FAMILY = {0: "dense_direct", 1: "dense_lds", 2: "dense_small", 3: "diag",
                 4: "wide", 5: "ucry", 6: "dense_bfly", 7: "dense_mfma"}
STATUS = {0: "SV_OK", 1: "SV_PENDING", -1: "SV_ERR_INVALID", -2: "SV_ERR_OOM",
          -3: "SV_ERR_HIP", -4: "SV_ERR_NOT_SYMMETRIC", -5: "SV_ERR_NOT_POSDEF",
          -6: "SV_ERR_SHAPE", -7: "SV_ERR_BUSY", -8: "SV_ERR_SINGULAR"}


class HHLSVError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.sv_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")


class HHLInfo(ctypes.Structure):
    _fields_ = [("n_sys", ctypes.c_int), ("n_clock", ctypes.c_int),
                ("n_total", ctypes.c_int), ("n_qpe_est", ctypes.c_int),
                ("n_gates", ctypes.c_int), ("dim", ctypes.c_int),
                ("j0", ctypes.c_int), ("t", ctypes.c_double),
                ("C", ctypes.c_double), ("lambda_lo", ctypes.c_double),
                ("lambda_hi", ctypes.c_double), ("kappa", ctypes.c_double),
                ("b_norm", ctypes.c_double), ("x_offset", ctypes.c_int),
                ("sign_qubit", ctypes.c_int), ("dilated", ctypes.c_int),
                ("preconditioned", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PFInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int),
                ("n_unknowns", ctypes.c_int), ("mismatch", ctypes.c_double),
                ("hhl_seconds", ctypes.c_double), ("history", ctypes.c_double * 64)]


class SolutionInfo(ctypes.Structure):
    _fields_ = [("scale", ctypes.c_double), ("p_anc1", ctypes.c_double),
                ("p_anc1_clock0", ctypes.c_double), ("max_imag", ctypes.c_double),
                ("pad_leak", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SvbTune(ctypes.Structure):
    _fields_ = [("k_max", ctypes.c_int), ("group_max", ctypes.c_int), ("wave_target", ctypes.c_int),
                ("resident_kib", ctypes.c_int), ("tuned", ctypes.c_int), ("ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_sz = ctypes.c_size_t


def _proto(name, *args):
    f = getattr(_lib, name)
    f.argtypes = list(args)
    f.restype = ctypes.c_int
    return f


_lib.sv_last_error.restype = ctypes.c_char_p
_proto("sv_create", ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp))
_proto("sv_create_from_buffer", _vp, _sz, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp))
_proto("sv_set_stream", _vp, _vp)
_proto("sv_device_buffer", _vp, ctypes.POINTER(_vp), ctypes.POINTER(_sz), ctypes.POINTER(_vp))
_proto("sv_destroy", _vp)
_proto("sv_reset", _vp)
_proto("sv_get_amplitudes", _vp, _sz, _sz, _vp)
_proto("sv_set_amplitudes", _vp, _sz, _sz, _vp)
_proto("sv_get_amplitudes_at", _vp, ctypes.POINTER(ctypes.c_uint64), _sz, _vp)
_proto("sv_norm2", _vp, _dp)
_proto("circuit_build_hhl", _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.POINTER(_vp))
_proto("circuit_build_hhl_ex", _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
       ctypes.POINTER(_vp))
_proto("circuit_create", ctypes.c_int, ctypes.POINTER(_vp))
_proto("circuit_add_gate", _vp, ctypes.c_int, _ip, ctypes.c_int, _dp, ctypes.c_int)
_proto("circuit_info", _vp, ctypes.POINTER(HHLInfo))
_proto("circuit_shape", _vp, _ip, _ip)
_proto("circuit_serialize", _vp, _vp, ctypes.POINTER(_sz))
_proto("fuse", _vp, ctypes.c_int, ctypes.POINTER(_vp))
_proto("sv_apply", _vp, _vp)
_proto("sv_apply_timed", _vp, _vp, _dp, _ip, ctypes.c_int)
_proto("sv_synchronize", _vp)
_proto("sv_postselect_solution", _vp, _vp, _dp, ctypes.c_int, ctypes.POINTER(SolutionInfo))
_proto("sv_postselect_solution_noalloc", _vp, _sz, ctypes.c_int, ctypes.c_int, _vp, _vp, _dp, ctypes.c_int,
       ctypes.POINTER(SolutionInfo))
_proto("circuit_destroy", _vp)
_proto("sv_solution_x", _dp, ctypes.c_int, ctypes.POINTER(SolutionInfo), _dp)
_proto("sv_debug_set_grid_cap", ctypes.c_int)
_proto("sv_debug_set_dense_mfma", ctypes.c_int)
_proto("sv_debug_set_pair0", ctypes.c_int)
_proto("sv_stream_probe", _vp, ctypes.c_int, _dp)
_proto("sv_qubit_estimate", ctypes.c_int, ctypes.c_double, ctypes.c_int, _ip, _ip, _ip)
_proto("pf_mismatch_jacobian", ctypes.c_int, ctypes.c_int, _ip, _ip, _dp, _dp, _dp, _ip, _dp, _dp, _dp, _dp,
       _dp, _dp, _dp, _dp, _ip)
_proto("pf_newton_hhl", ctypes.c_int, ctypes.c_int, _ip, _ip, _dp, _dp, _dp, _ip, _dp, _dp, _dp, ctypes.c_int,
       ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp, ctypes.POINTER(PFInfo))
_proto("svb_create", ctypes.c_int, ctypes.c_int, _vp, ctypes.POINTER(_vp))
_proto("svb_add", _vp, _vp, _ip)
_proto("svb_run", _vp)
_proto("svb_solution", _vp, ctypes.c_int, _dp, ctypes.c_int, ctypes.POINTER(SolutionInfo))
_proto("svb_last_run_ms", _vp, _dp)
_proto("svb_run_timed", _vp, ctypes.c_int, _ip, _ip, _ip, _ip, _ip, _dp)
_proto("svb_run_timed_ops", _vp, ctypes.c_int, _ip, _ip, _ip, _ip, _ip, _dp)
_proto("svb_postselected", _vp, ctypes.c_int, _dp, ctypes.c_int, _dp)
_proto("svb_size", _vp, _ip)
_proto("svb_destroy", _vp)
_proto("svb_autotune", ctypes.c_int, _vp, ctypes.c_int, _ip, _dp)
_proto("svb_autotune_ex", ctypes.c_int, _vp, ctypes.c_int, ctypes.POINTER(SvbTune), _dp)
_proto("svb_get_tune", ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(SvbTune))
_proto("svb_set_tune", ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(SvbTune))
_u64 = ctypes.c_uint64
_proto("svs_start", _sz, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp))
_proto("svs_configure", _vp, ctypes.c_int, ctypes.c_double)
_proto("svs_submit", _vp, _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.POINTER(_u64))
_proto("svs_poll", _vp, _u64, _dp, ctypes.c_int, ctypes.POINTER(SolutionInfo))
_proto("svs_poll_ex", _vp, _u64, _dp, ctypes.c_int, ctypes.POINTER(SolutionInfo), _dp, ctypes.c_int, _dp)
_proto("svs_cancel", _vp, _u64)
_proto("svs_drain", _vp, ctypes.c_double)
_proto("svs_stats", _vp, _dp, _dp, _dp, ctypes.POINTER(_u64))
_proto("svs_counts", _vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64), ctypes.POINTER(_u64))
_proto("svs_stop", _vp)
_proto("svs_profile", _vp, _dp, ctypes.c_int)


def _check(rc, where):
    if rc not in (0, 1):
        raise HHLSVError(rc, where)
    return rc


def _dptr(a):
    return a.ctypes.data_as(_dp)


def _amp_dtype(dtype):
    return np.complex128 if DTYPES[dtype] == C128 else np.complex64


# ------------------------------------------------------------------ circuits
class Circuit:
    """Owning wrapper of an ``sv_circuit*``."""

    def __init__(self, handle):
        self.handle = _vp(handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            _lib.circuit_destroy(h)
            self.handle = _vp()

    @property
    def shape(self):
        n = ctypes.c_int()
        g = ctypes.c_int()
        _check(_lib.circuit_shape(self.handle, ctypes.byref(n), ctypes.byref(g)), "circuit_shape")
        return n.value, g.value

    @property
    def n_qubits(self):
        return self.shape[0]

    @property
    def n_gates(self):
        return self.shape[1]

    def info(self):
        out = HHLInfo()
        _check(_lib.circuit_info(self.handle, ctypes.byref(out)), "circuit_info")
        return out.as_dict()

    def serialize(self) -> bytes:
        ln = _sz()
        _check(_lib.circuit_serialize(self.handle, None, ctypes.byref(ln)), "circuit_serialize")
        buf = ctypes.create_string_buffer(ln.value)
        _check(_lib.circuit_serialize(self.handle, buf, ctypes.byref(ln)), "circuit_serialize")
        return buf.raw[: ln.value]

    def gates(self):
        """Decode the serialised gate list: [(kind_name, qubits, params)]."""
        raw = self.serialize()
        n, ng = np.frombuffer(raw, dtype="<i4", count=2)
        off = 8
        out = []
        for _ in range(int(ng)):
            kind, nq, npar = np.frombuffer(raw, dtype="<i4", count=3, offset=off)
            off += 12
            qs = np.frombuffer(raw, dtype="<i4", count=int(nq), offset=off).tolist()
            off += 4 * int(nq)
            ps = np.frombuffer(raw, dtype="<f8", count=int(npar), offset=off).copy()
            off += 8 * int(npar)
            out.append((KIND_NAME[int(kind)], qs, ps))
        return out


def circuit_create(n_qubits: int) -> Circuit:
    h = _vp()
    _check(_lib.circuit_create(n_qubits, ctypes.byref(h)), "circuit_create")
    return Circuit(h.value)


def circuit_add_gate(c: Circuit, kind, qubits, params=()):
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).ravel())
    k = KIND[kind] if isinstance(kind, str) else int(kind)
    _check(_lib.circuit_add_gate(c.handle, k, q.ctypes.data_as(_ip), q.size,
                                 _dptr(p) if p.size else None, p.size), "circuit_add_gate")


def circuit_from_gates(n_qubits: int, gates) -> Circuit:
    """Generic circuit from ``workloads.Gate`` tuples (kind, qubits, params)."""
    c = circuit_create(n_qubits)
    for g in gates:
        circuit_add_gate(c, g[0], g[1], g[2])
    return c


SV_HHL_DEVICE_EVOLUTIONS = 1
SV_HHL_SIGNED = 2
SV_HHL_DILATE = 4
SV_HHL_AUTO = 8
SV_HHL_GAUSS_SEIDEL = 16
HHL_MODES = {"spd": 0, "signed": SV_HHL_SIGNED, "dilate": SV_HHL_DILATE, "auto": SV_HHL_AUTO,
             "gauss_seidel": SV_HHL_GAUSS_SEIDEL}


def _hhl_flags(mode: str) -> int:
    try:
        return HHL_MODES[mode]
    except KeyError:
        raise ValueError(f"mode must be one of {sorted(HHL_MODES)}") from None


def circuit_build_hhl(A, b, clock_bits: int, t: float = 0.0,
                      device_evolutions: bool = False, mode: str = "spd") -> Circuit:
    """HHL circuit for A x = b.  device_evolutions=True keeps the
    eigen-decomposition and builds the controlled e^{iAt 2^j} on the GPU.
    mode: "spd" (symmetric, positive on b's span), "signed" (sign qubit),
    "dilate" (general square A through [[0, A'], [A'^T, 0]]), "auto", or
    "gauss_seidel" (left Gauss-Seidel preconditioning, then the dilation)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64).ravel()
    if A.shape != (b.size, b.size):
        raise ValueError("A must be dim x dim with dim = len(b)")
    h = _vp()
    flags = (SV_HHL_DEVICE_EVOLUTIONS if device_evolutions else 0) | _hhl_flags(mode)
    _check(_lib.circuit_build_hhl_ex(_dptr(A), _dptr(b), b.size, clock_bits, float(t), flags,
                                     ctypes.byref(h)), "circuit_build_hhl")
    return Circuit(h.value)


def fuse(c: Circuit, k_max: int) -> Circuit:
    h = _vp()
    _check(_lib.fuse(c.handle, k_max, ctypes.byref(h)), "fuse")
    return Circuit(h.value)


def sv_qubit_estimate(dim: int, kappa: float, has_negative: bool):
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(_lib.sv_qubit_estimate(dim, kappa, int(has_negative), ctypes.byref(a),
                                  ctypes.byref(b), ctypes.byref(c)), "sv_qubit_estimate")
    return a.value, b.value, c.value


# -------------------------------------------------------------------- states
class State:
    """Owning wrapper of an ``sv_state*`` (device state vector + stream)."""

    def __init__(self, handle, n, dtype, keepalive=None):
        self.handle = _vp(handle)
        self.n = n
        self.dtype = DTYPES[dtype]
        self._keepalive = keepalive

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            _lib.sv_destroy(h)
            self.handle = _vp()

    def close(self):
        self.__del__()

    @classmethod
    def from_tensor(cls, tensor, n_qubits: int, dtype="c128"):
        """Adopt a torch CUDA tensor's memory (kept alive by the state)."""
        h = _vp()
        nbytes = tensor.numel() * tensor.element_size()
        _check(_lib.sv_create_from_buffer(_vp(tensor.data_ptr()), nbytes, n_qubits,
                                          DTYPES[dtype], ctypes.byref(h)), "sv_create_from_buffer")
        return cls(h.value, n_qubits, dtype, keepalive=tensor)

    def set_stream(self, stream=None):
        """Order work on a torch stream (or a raw hipStream_t integer)."""
        ptr = getattr(stream, "cuda_stream", stream)
        _check(_lib.sv_set_stream(self.handle, _vp(ptr) if ptr else None), "sv_set_stream")

    def reset(self):
        _check(_lib.sv_reset(self.handle), "sv_reset")

    def device_buffer(self):
        """(device address, bytes, hipStream_t) of the state's amplitudes."""
        p, nb, st = _vp(), _sz(), _vp()
        _check(_lib.sv_device_buffer(self.handle, ctypes.byref(p), ctypes.byref(nb), ctypes.byref(st)),
               "sv_device_buffer")
        return p.value, nb.value, st.value

    def get(self, offset: int = 0, count: int | None = None) -> np.ndarray:
        if count is None:
            count = (1 << self.n) - offset
        out = np.empty(count, dtype=_amp_dtype(self.dtype))
        _check(_lib.sv_get_amplitudes(self.handle, offset, count, out.ctypes.data_as(_vp)),
               "sv_get_amplitudes")
        return out

    def set(self, values, offset: int = 0):
        v = np.ascontiguousarray(values, dtype=_amp_dtype(self.dtype))
        _check(_lib.sv_set_amplitudes(self.handle, offset, v.size, v.ctypes.data_as(_vp)),
               "sv_set_amplitudes")

    def get_at(self, indices) -> np.ndarray:
        idx = np.ascontiguousarray(indices, dtype=np.uint64)
        out = np.empty(idx.size, dtype=_amp_dtype(self.dtype))
        _check(_lib.sv_get_amplitudes_at(self.handle,
                                         idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                         idx.size, out.ctypes.data_as(_vp)), "sv_get_amplitudes_at")
        return out

    def norm2(self) -> float:
        out = ctypes.c_double()
        _check(_lib.sv_norm2(self.handle, ctypes.byref(out)), "sv_norm2")
        return out.value

    def apply(self, c: Circuit):
        _check(_lib.sv_apply(self.handle, c.handle), "sv_apply")

    def apply_timed(self, c: Circuit):
        """Apply and time every launch: (ms per gate, kernel family per gate)."""
        ng = c.n_gates
        ms = np.zeros(max(ng, 1))
        fam = np.zeros(max(ng, 1), dtype=np.int32)
        _check(_lib.sv_apply_timed(self.handle, c.handle, _dptr(ms), fam.ctypes.data_as(_ip),
                                   ms.size), "sv_apply_timed")
        return ms[:ng], fam[:ng]

    def synchronize(self):
        _check(_lib.sv_synchronize(self.handle), "sv_synchronize")

    def stream_probe(self, reps: int = 5) -> np.ndarray:
        """Device ms of each of ``reps`` in-place read/write-back launches
        with the dense sweeps' access shape (complex128, n >= 10)."""
        ms = np.zeros(reps)
        _check(_lib.sv_stream_probe(self.handle, reps, _dptr(ms)), "sv_stream_probe")
        return ms

    def postselect_solution(self, hhl: Circuit, dim: int):
        x = np.zeros(dim)
        info = SolutionInfo()
        _check(_lib.sv_postselect_solution(self.handle, hhl.handle, _dptr(x), dim,
                                           ctypes.byref(info)), "sv_postselect_solution")
        return x, info.as_dict()


def sv_create(n_qubits: int, dtype="c128") -> State:
    h = _vp()
    _check(_lib.sv_create(n_qubits, DTYPES[dtype], ctypes.byref(h)), "sv_create")
    return State(h.value, n_qubits, dtype)


def sv_apply(s: State, c: Circuit):
    s.apply(c)


def sv_postselect_solution(s: State, hhl: Circuit, dim: int):
    return s.postselect_solution(hhl, dim)


def sv_postselect_solution_noalloc(dev_ptr: int, nbytes: int, n_qubits: int, dtype, stream,
                                   hhl: Circuit, dim: int):
    """The readout of sv_postselect_solution on caller-owned device memory
    (a raw device address of 2^n_qubits amplitudes), with no allocation in
    the library.  stream: a torch stream or a raw hipStream_t integer."""
    ptr = getattr(stream, "cuda_stream", stream)
    x = np.zeros(dim)
    info = SolutionInfo()
    _check(_lib.sv_postselect_solution_noalloc(_vp(dev_ptr), nbytes, n_qubits, DTYPES[dtype],
                                               _vp(ptr) if ptr else None, hhl.handle, _dptr(x), dim,
                                               ctypes.byref(info)), "sv_postselect_solution_noalloc")
    return x, info.as_dict()


def solve(A, b, clock_bits: int, dtype="c128", k_max: int | None = None, t: float = 0.0,
          mode: str = "spd"):
    """One HHL solve end to end: build, (fuse), apply, postselect.

    Returns (x, x_hat, solution_info, hhl_info)."""
    c = circuit_build_hhl(A, b, clock_bits, t, mode=mode)
    run = fuse(c, k_max) if k_max else c
    s = sv_create(c.n_qubits, dtype)
    s.apply(run)
    x_hat, info = s.postselect_solution(c, len(b))
    return sv_solution_x(x_hat, info), x_hat, info, c.info()


def sv_solution_x(x_hat, info: dict) -> np.ndarray:
    """Step 4b, in the library: x = scale * x_hat."""
    x_hat = np.ascontiguousarray(x_hat, dtype=np.float64)
    si = SolutionInfo(**{k: float(info[k]) for k, _ in SolutionInfo._fields_})
    x = np.zeros(x_hat.size)
    _check(_lib.sv_solution_x(_dptr(x_hat), x_hat.size, ctypes.byref(si), _dptr(x)), "sv_solution_x")
    return x


def sv_debug_set_grid_cap(max_workgroups: int):
    """Test hook: bound every launch's workgroup count (0 = no bound)."""
    _check(_lib.sv_debug_set_grid_cap(int(max_workgroups)), "sv_debug_set_grid_cap")


def sv_debug_set_dense_mfma(enable):
    """Matrix-core form of 4/5-qubit dense gates: True or 1 (default rules),
    False or 0 (vector forms), 2 (also every other 4-qubit gate it can take)."""
    _check(_lib.sv_debug_set_dense_mfma(int(enable)), "sv_debug_set_dense_mfma")


def sv_debug_set_pair0(enable: bool):
    """complex64 gates with bit 0 the only target inside a line: pair kernel
    (True, default) or LDS regroup (False)."""
    _check(_lib.sv_debug_set_pair0(int(bool(enable))), "sv_debug_set_pair0")


# ------------------------------------------------------------------- batches
class Batch:
    """Owning wrapper of an ``svb*``: many small HHL solves per launch."""

    def __init__(self, dtype="c128", k_max: int = 0, stream=None):
        h = _vp()
        ptr = getattr(stream, "cuda_stream", stream)
        _check(_lib.svb_create(DTYPES[dtype], k_max, _vp(ptr) if ptr else None, ctypes.byref(h)),
               "svb_create")
        self.handle = h
        self.dims = []
        self.ns = []

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            _lib.svb_destroy(h)
            self.handle = _vp()

    def close(self):
        self.__del__()

    def add(self, hhl: Circuit) -> int:
        idx = ctypes.c_int()
        _check(_lib.svb_add(self.handle, hhl.handle, ctypes.byref(idx)), "svb_add")
        inf = hhl.info()
        self.dims.append(inf["dim"])
        self.ns.append(inf["n_sys"])
        return idx.value

    def __len__(self):
        return len(self.dims)

    def run(self) -> float:
        """Run every instance; returns the device time in ms."""
        _check(_lib.svb_run(self.handle), "svb_run")
        ms = ctypes.c_double()
        _check(_lib.svb_last_run_ms(self.handle, ctypes.byref(ms)), "svb_last_run_ms")
        return ms.value

    def run_timed(self, cap: int = 4096):
        """Eager run, one work item after another, each timed: a list of
        dicts (kind "batched" or "swept", n, count, ops, ms)."""
        items = ctypes.c_int()
        kind, n, count, ops = (np.zeros(cap, dtype=np.int32) for _ in range(4))
        ms = np.zeros(cap)
        _check(_lib.svb_run_timed(self.handle, cap, ctypes.byref(items), kind.ctypes.data_as(_ip),
                                  n.ctypes.data_as(_ip), count.ctypes.data_as(_ip), ops.ctypes.data_as(_ip),
                                  _dptr(ms)), "svb_run_timed")
        return [{"kind": "swept" if kind[i] else "batched", "n": int(n[i]), "count": int(count[i]),
                 "ops": int(ops[i]), "ms": float(ms[i])} for i in range(items.value)]

    def run_timed_ops(self, cap: int = 65536):
        """Each fused op of the grouped sweeps timed on its own: a list of
        dicts (item, family, k, controls, ms); run() afterwards for results."""
        count = ctypes.c_int()
        item, fam, k, ctl = (np.zeros(cap, dtype=np.int32) for _ in range(4))
        ms = np.zeros(cap)
        _check(_lib.svb_run_timed_ops(self.handle, cap, ctypes.byref(count), item.ctypes.data_as(_ip),
                                      fam.ctypes.data_as(_ip), k.ctypes.data_as(_ip), ctl.ctypes.data_as(_ip),
                                      _dptr(ms)), "svb_run_timed_ops")
        return [{"item": int(item[i]), "family": KERNEL_FAMILY[int(fam[i])], "k": int(k[i]),
                 "controls": int(ctl[i]), "ms": float(ms[i])} for i in range(count.value)]

    def solution(self, index: int):
        dim = self.dims[index]
        x = np.zeros(dim)
        info = SolutionInfo()
        _check(_lib.svb_solution(self.handle, index, _dptr(x), dim, ctypes.byref(info)),
               "svb_solution")
        return x, info.as_dict()


    def postselected(self, index: int, count: int | None = None):
        """Raw postselected block y (complex, count <= 2^ns entries) and
        P(ancilla = 1) of one instance."""
        ns = self.ns[index]
        count = (1 << ns) if count is None else count
        y = np.zeros(2 * count)
        p1 = ctypes.c_double()
        _check(_lib.svb_postselected(self.handle, index, _dptr(y), count, ctypes.byref(p1)),
               "svb_postselected")
        return y.view(np.complex128), p1.value


def svb_autotune_ex(dtype, sample: Circuit, copies: int = 64):
    """Tune every launch choice for the sample's shape (see svb_autotune_ex in
    hhlsv.h); returns (choice dict, device ms per k = 1..5)."""
    t = SvbTune()
    ms = np.zeros(5)
    _check(_lib.svb_autotune_ex(DTYPES[dtype], sample.handle, copies, ctypes.byref(t), _dptr(ms)),
           "svb_autotune_ex")
    return t.as_dict(), ms


def svb_get_tune(dtype, ns: int, m: int) -> dict:
    t = SvbTune()
    _check(_lib.svb_get_tune(DTYPES[dtype], ns, m, ctypes.byref(t)), "svb_get_tune")
    return t.as_dict()


def svb_set_tune(dtype, ns: int, m: int, k_max: int = 3, group_max: int = 256, wave_target: int = 1024,
                 resident_kib: int = 64):
    t = SvbTune(k_max, group_max, wave_target, resident_kib, 0, 0.0)
    _check(_lib.svb_set_tune(DTYPES[dtype], ns, m, ctypes.byref(t)), "svb_set_tune")


def svb_autotune(dtype, sample: Circuit, copies: int = 64):
    """Time k_max = 1..5 on copies of ``sample``; record and return the best."""
    best = ctypes.c_int()
    ms = np.zeros(5)
    _check(_lib.svb_autotune(DTYPES[dtype], sample.handle, copies, ctypes.byref(best), _dptr(ms)),
           "svb_autotune")
    return best.value, ms


# ------------------------------------------------------------------- serving
SVS_OPT = {"prep_threads": 1, "k_max": 2, "max_batch": 3, "streams": 4, "queue_limit": 5,
           "fail_alloc_at": 6, "batch_max_qubits": 7, "hhl_flags": 8, "launchers": 9,
           "group_window_us": 10, "lds_max_qubits": 11}


class Server:
    """Owning wrapper of an ``svs*`` continuous-batching server."""

    def __init__(self, dtype="c128", hbm_budget_bytes: int = 0, max_slots: int = 4096,
                 mode: str = "spd", **options):
        h = _vp()
        _check(_lib.svs_start(hbm_budget_bytes, max_slots, DTYPES[dtype], ctypes.byref(h)), "svs_start")
        self.handle = h
        self.dims = {}
        if mode != "spd":
            options = dict(options, hhl_flags=_hhl_flags(mode))
        for k, v in options.items():
            _check(_lib.svs_configure(self.handle, SVS_OPT[k], float(v)), "svs_configure")

    def submit(self, A, b, clock_bits: int, t: float = 0.0) -> int:
        A = np.ascontiguousarray(A, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64).ravel()
        tk = _u64()
        _check(_lib.svs_submit(self.handle, _dptr(A), _dptr(b), b.size, clock_bits, float(t),
                               ctypes.byref(tk)), "svs_submit")
        self.dims[tk.value] = b.size
        return tk.value

    def poll(self, ticket: int):
        """None while pending; (x_hat, info) when done; raises on failure."""
        dim = self.dims[ticket]
        x = np.zeros(dim)
        info = SolutionInfo()
        rc = _lib.svs_poll(self.handle, ticket, _dptr(x), dim, ctypes.byref(info))
        if rc == 1:
            return None
        self.dims.pop(ticket, None)
        _check(rc, "svs_poll")
        return x, info.as_dict()

    def poll_ex(self, ticket: int, y_count: int):
        """As poll, plus the raw postselected block y (y_count complex
        entries) and P(ancilla = 1): None while pending, else
        (x_hat, info, y, p_anc1)."""
        dim = self.dims[ticket]
        x = np.zeros(dim)
        y = np.zeros(2 * y_count)
        p1 = ctypes.c_double()
        info = SolutionInfo()
        rc = _lib.svs_poll_ex(self.handle, ticket, _dptr(x), dim, ctypes.byref(info), _dptr(y), y_count,
                              ctypes.byref(p1))
        if rc == 1:
            return None
        self.dims.pop(ticket, None)
        _check(rc, "svs_poll_ex")
        return x, info.as_dict(), y.view(np.complex128), p1.value

    def cancel(self, ticket: int):
        _check(_lib.svs_cancel(self.handle, ticket), "svs_cancel")

    def drain(self, timeout_s: float = 0.0):
        _check(_lib.svs_drain(self.handle, timeout_s), "svs_drain")

    def stats(self):
        p50, p99, sps = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        rej = _u64()
        _check(_lib.svs_stats(self.handle, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(sps),
                              ctypes.byref(rej)), "svs_stats")
        done, failed, pending = _u64(), _u64(), _u64()
        _check(_lib.svs_counts(self.handle, ctypes.byref(done), ctypes.byref(failed),
                               ctypes.byref(pending)), "svs_counts")
        return {"p50_s": p50.value, "p99_s": p99.value, "solves_per_s": sps.value,
                "rejected": rej.value, "done": done.value, "failed": failed.value,
                "pending": pending.value}

    def profile(self):
        v = np.zeros(10)
        _check(_lib.svs_profile(self.handle, _dptr(v), 10), "svs_profile")
        keys = ["queue_s", "prep_s", "upload_s", "ready_wait_s", "gpu_s", "batched", "alone", "prep_threads",
                "groups", "grouped"]
        return dict(zip(keys, v.tolist()))

    def stop(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            _lib.svs_stop(h)
            self.handle = _vp()

    def __del__(self):
        self.stop()


# ---------------------------------------------------------------- power flow
def _pf_arrays(case):
    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    return (i32(case["from"]), i32(case["to"]), f64(case["r"]), f64(case["x"]), f64(case["bsh"]),
            i32(case["type"]), f64(case["p"]), f64(case["q"]), f64(case["vset"]))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def pf_mismatch_jacobian(case, vm, va):
    """(P, Q, F, J) of the AC power-flow model at magnitudes vm, angles va."""
    fr, to, r, x, b, ty, p, q, vs = _pf_arrays(case)
    nb = ty.size
    vm = np.ascontiguousarray(vm, dtype=np.float64)
    va = np.ascontiguousarray(va, dtype=np.float64)
    nu = ctypes.c_int()
    _check(_lib.pf_mismatch_jacobian(nb, fr.size, _iptr(fr), _iptr(to), _dptr(r), _dptr(x), _dptr(b),
                                     _iptr(ty), None, None, None, None, None, None, None, None,
                                     ctypes.byref(nu)), "pf_mismatch_jacobian")
    N = nu.value
    P, Q, F, J = np.zeros(nb), np.zeros(nb), np.zeros(N), np.zeros((N, N))
    _check(_lib.pf_mismatch_jacobian(nb, fr.size, _iptr(fr), _iptr(to), _dptr(r), _dptr(x), _dptr(b),
                                     _iptr(ty), _dptr(p), _dptr(q), _dptr(vm), _dptr(va), _dptr(P), _dptr(Q),
                                     _dptr(F), _dptr(J), None), "pf_mismatch_jacobian")
    return P, Q, F, J


def pf_newton(case, clock_bits: int, mode: str = "dilate", dtype="c128", k_max: int = 3,
              max_iter: int = 30, tol: float = 1e-9, device_evolutions: bool = False):
    """Newton-Raphson AC power flow with HHL inner solves on the GPU.
    mode: "dilate", "gauss_seidel" or "auto".  Returns (vm, va, info dict)."""
    fr, to, r, x, b, ty, p, q, vs = _pf_arrays(case)
    nb = ty.size
    vm, va = np.zeros(nb), np.zeros(nb)
    flags = _hhl_flags(mode) | (SV_HHL_DEVICE_EVOLUTIONS if device_evolutions else 0)
    info = PFInfo()
    _check(_lib.pf_newton_hhl(nb, fr.size, _iptr(fr), _iptr(to), _dptr(r), _dptr(x), _dptr(b), _iptr(ty),
                              _dptr(p), _dptr(q), _dptr(vs), clock_bits, flags, DTYPES[dtype], k_max, max_iter,
                              float(tol), _dptr(vm), _dptr(va), ctypes.byref(info)), "pf_newton_hhl")
    d = {"iterations": info.iterations, "converged": bool(info.converged), "n_unknowns": info.n_unknowns,
         "mismatch": info.mismatch, "hhl_seconds": info.hhl_seconds,
         "history": list(info.history[:min(info.iterations + 1, 64)])}
    return vm, va, d
