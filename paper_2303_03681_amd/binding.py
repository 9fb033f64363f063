"""Thin Python binding of the C ABI in include/mps.h (argument marshalling only).

Every numerical step runs in the HIP library libmps_hip.so; this module only
converts numpy arrays to pointers and status codes to exceptions.  If the
library has not been built, loading fails loudly -- there is no fallback.

torch is imported (when installed) before the library is loaded so that the
process holds a single HIP runtime: the library then binds to the runtime
torch already loaded, and torch streams can be handed to it.
"""

from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG_DIR, "libmps_hip.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG_DIR), "include", "mps.h")

STATUS = {
    0: "MPS_OK", -1: "MPS_ERR_ARG", -2: "MPS_ERR_OOM", -3: "MPS_ERR_BUDGET",
    -4: "MPS_ERR_NOCONV", -5: "MPS_ERR_NONFINITE", -6: "MPS_ERR_DEVICE", -7: "MPS_ERR_STATE",
}
PREC = {"c128": 0, "c64": 1, "split_bf16": 2, "split_f16": 3}


class MpsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class _Config(C.Structure):
    _fields_ = [
        ("n_qubits", C.c_int32),
        ("max_bond", C.c_int32),
        ("svd_cutoff", C.c_double),
        ("max_jacobi_sweeps", C.c_int32),
        ("init_bits", C.c_void_p),
        ("stream", C.c_void_p),
        ("hbm_budget_bytes", C.c_size_t),
    ]


class Timing(C.Structure):
    _fields_ = [
        ("env_ms", C.c_double),
        ("env_launches", C.c_int64),
        ("env_flops", C.c_double),
        ("env_updates", C.c_int64),
        ("close_ms", C.c_double),
        ("close_flops", C.c_double),
        ("expect_ms", C.c_double),
        ("gates_ms", C.c_double),
        ("canon_ms", C.c_double),
        ("jacobi_sweeps", C.c_int64),
        ("jacobi_ms", C.c_double),
        ("jacobi_flops", C.c_double),
        ("graph_launches", C.c_int64),
        ("jacobi_batch_sweeps", C.c_int64),
        ("jacobi_multi_items", C.c_int64),
        ("jacobi_wide_items", C.c_int64),
        ("jacobi_split_batches", C.c_int64),
        ("close_tile_flops", C.c_double),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None

_P = C.c_void_p
_I32 = C.c_int32
_I64 = C.c_int64
_D = C.c_double

_SIGS = {
    "mps_create": [_P, _P],
    "mps_destroy": [_P],
    "mps_reset": [_P, _P],
    "mps_apply_gate": [_P, _I32, _I32, _P],
    "mps_apply_gates": [_P, _I64, _P, _P, _P, _P],
    "mps_canonicalize": [_P],
    "mps_norm": [_P, _P],
    "mps_discarded_weight": [_P, _P],
    "mps_bond_dims": [_P, _P],
    "mps_pauli_sum_create": [_I32, _I64, _P, _P, _P],
    "mps_pauli_sum_destroy": [_P],
    "mps_pauli_sum_stats": [_P, _P, _P, _P, _P],
    "mps_pauli_sum_export": [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "mps_expect_pauli_sum": [_P, _P, C.c_int, _P, _P],
    "mps_export": [_P, _I32, _P, _P, _P, _P],
    "mps_import": [_P, _I32, _I32, _I32, _P, _P],
    "mps_jacobi_svd": [_I32, _I32, _P, _P, _P, _P],
    "mps_set_timing": [_P, _I32],
    "mps_set_fused_gates": [_P, _I32],
    "mps_set_jacobi_groups": [_P, _I32],
    "mps_set_autotune": [_P, _I32],
    "mps_autotune_table": [_P, _I64, _P],
    "mps_autotune_reset": [],
    "mps_set_env_tile": [_P, _I32],
    "mps_set_graphs": [_P, _I32],
    "mps_copy": [_P, _P],
    "mps_expect_pauli_rows": [_P, _P, C.c_int, _I64, _P, _P, _P, _P],
    "mps_apply_gates_multi": [_I32, _P, _P, _P, _P, _P, _P, _P],
    "mps_get_timing": [_P, _P],
    "mps_device_bytes": [_P, _P],
    "mps_selftest_mfma": [_P],
    "mps_expect_pauli_sums": [_P, _I32, _P, C.c_int, _P, _P],
    "mps_expect_pauli_sum_multi": [_I32, _P, _P, C.c_int, _P, _P],
    "mps_to_statevector": [_P, _P],
    "mps_jacobi_svd_noalloc": [_I32, _I32, _P, _P, _P, _P, _P],
}


def header_symbols() -> list[str]:
    """Entry points declared in include/mps.h."""
    text = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"\b(mps_[a-z0-9_]+)\s*\(", text)))


def load():
    """Load libmps_hip.so (once); raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    try:  # share torch's HIP runtime when torch is present
        import torch  # noqa: F401
    except Exception:
        pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run python -m paper_2303_03681_amd.build)")
    lib = C.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.mps_last_error.argtypes = []
    lib.mps_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(st: int):
    if st != 0:
        msg = _lib.mps_last_error().decode(errors="replace")
        raise MpsError(st, msg)


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _cplx(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


class PauliSum:
    """A compiled, device-independent plan for sum_k coeffs[k] P_k."""

    def __init__(self, codes: np.ndarray, coeffs: np.ndarray):
        lib = load()
        codes = np.ascontiguousarray(codes, dtype=np.uint8)
        coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
        if codes.ndim != 2 or codes.shape[0] != coeffs.shape[0]:
            raise ValueError("codes must be (T, N) and coeffs (T,)")
        self.n_qubits = int(codes.shape[1])
        self.n_terms = int(codes.shape[0])
        h = C.c_void_p()
        _check(lib.mps_pauli_sum_create(self.n_qubits, self.n_terms, _ptr(codes), _ptr(coeffs),
                                        C.byref(h)))
        self._h = h

    def stats(self) -> dict:
        nl, nr, nc = C.c_int64(), C.c_int64(), C.c_int64()
        meet = C.c_int32()
        _check(_lib.mps_pauli_sum_stats(self._h, C.byref(nl), C.byref(nr), C.byref(nc),
                                        C.byref(meet)))
        return {"left_updates": nl.value, "right_updates": nr.value, "closes": nc.value,
                "meet_bond": meet.value}

    def export(self) -> dict:
        """Plan arrays (host logic inspection): trie nodes and per-term closes."""
        st = self.stats()
        nl, nr, T = st["left_updates"], st["right_updates"], self.n_terms
        lpar = np.zeros(nl, np.int32)
        lsite = np.zeros(nl, np.int32)
        llet = np.zeros(nl, np.int32)
        rpar = np.zeros(nr, np.int32)
        rsite = np.zeros(nr, np.int32)
        rlet = np.zeros(nr, np.int32)
        cb = np.zeros(T, np.int32)
        cl = np.zeros(T, np.int32)
        cr = np.zeros(T, np.int32)
        _check(_lib.mps_pauli_sum_export(self._h, _ptr(lpar), _ptr(lsite), _ptr(llet), _ptr(rpar),
                                         _ptr(rsite), _ptr(rlet), _ptr(cb), _ptr(cl), _ptr(cr)))
        return {"left": (lpar, lsite, llet), "right": (rpar, rsite, rlet),
                "close": (cb, cl, cr), "meet": st["meet_bond"]}

    def close(self):
        if getattr(self, "_h", None):
            _lib.mps_pauli_sum_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mps:
    """Handle on a device-resident MPS (see include/mps.h)."""

    def __init__(self, n_qubits: int, max_bond: int, cutoff: float = 1e-14, bits=None,
                 stream: int | None = None, hbm_budget_bytes: int = 0, max_jacobi_sweeps: int = 0):
        lib = load()
        self.n = int(n_qubits)
        self._bits = None if bits is None else np.ascontiguousarray(bits, dtype=np.uint8)
        cfg = _Config(self.n, int(max_bond), float(cutoff), int(max_jacobi_sweeps),
                      None if self._bits is None else self._bits.ctypes.data, stream,
                      int(hbm_budget_bytes))
        h = C.c_void_p()
        _check(lib.mps_create(C.byref(cfg), C.byref(h)))
        self._h = h

    # -- state ------------------------------------------------------------
    def reset(self, bits=None):
        b = None if bits is None else np.ascontiguousarray(bits, dtype=np.uint8)
        _check(_lib.mps_reset(self._h, _ptr(b)))

    def apply_gate(self, q0: int, q1: int, u):
        m = _cplx(u)
        _check(_lib.mps_apply_gate(self._h, int(q0), int(q1), _ptr(m.view(np.float64))))

    def apply_gates(self, q0, q1, u_packed) -> int:
        """u_packed: (G, 16, 2) float64 (re, im) as built by workloads.pack_gates."""
        q0 = np.ascontiguousarray(q0, dtype=np.int32)
        q1 = np.ascontiguousarray(q1, dtype=np.int32)
        u = np.ascontiguousarray(u_packed, dtype=np.float64)
        if u.size != 32 * q0.size or q1.size != q0.size:
            raise ValueError("u_packed must hold 32 doubles per gate")
        done = C.c_int64()
        try:
            _check(_lib.mps_apply_gates(self._h, q0.size, _ptr(q0), _ptr(q1), _ptr(u), C.byref(done)))
        except MpsError as err:
            err.n_done = done.value  # gates applied before the failure
            raise
        return done.value

    def canonicalize(self):
        _check(_lib.mps_canonicalize(self._h))

    def norm(self) -> float:
        v = C.c_double()
        _check(_lib.mps_norm(self._h, C.byref(v)))
        return v.value

    def discarded_weight(self) -> float:
        v = C.c_double()
        _check(_lib.mps_discarded_weight(self._h, C.byref(v)))
        return v.value

    def bond_dims(self) -> np.ndarray:
        d = np.zeros(self.n + 1, np.int32)
        _check(_lib.mps_bond_dims(self._h, _ptr(d)))
        return d

    def export_site(self, q: int):
        dl, dr = C.c_int32(), C.c_int32()
        _check(_lib.mps_export(self._h, int(q), C.byref(dl), C.byref(dr), None, None))
        b = np.zeros((2, dl.value, dr.value), np.complex128)
        lam = np.zeros(dl.value, np.float64)
        _check(_lib.mps_export(self._h, int(q), C.byref(dl), C.byref(dr),
                               _ptr(b.view(np.float64)), _ptr(lam)))
        return b, lam

    def import_site(self, q: int, b, lam_left):
        b = _cplx(b)
        lam = np.ascontiguousarray(lam_left, dtype=np.float64)
        _check(_lib.mps_import(self._h, int(q), b.shape[1], b.shape[2],
                               _ptr(b.view(np.float64)), _ptr(lam)))

    # -- expectations -------------------------------------------------------
    def expect_rows(self, psum: PauliSum, row_ptr, cols, vals, prec: str = "c128") -> np.ndarray:
        """out[r] = sum over row r of vals[i] * Re<P_cols[i]> (CSR rows)."""
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        vals = np.ascontiguousarray(vals, dtype=np.float64)
        n_rows = row_ptr.size - 1
        out = np.zeros(max(n_rows, 0), np.float64)
        _check(_lib.mps_expect_pauli_rows(self._h, psum._h, PREC[prec], n_rows, _ptr(row_ptr), _ptr(cols),
                                          _ptr(vals), _ptr(out)))
        return out

    def expect(self, psum: PauliSum, prec: str = "c128", per_term: bool = False):
        e = C.c_double()
        out = np.zeros(psum.n_terms, np.float64) if per_term else None
        _check(_lib.mps_expect_pauli_sum(self._h, psum._h, PREC[prec], C.byref(e), _ptr(out)))
        return (e.value, out) if per_term else e.value

    def expect_chunks(self, plans, prec: str = "c128", per_term: bool = False):
        """E over several plans (chunks of one Pauli sum), summed on the device."""
        n = len(plans)
        arr = (C.c_void_p * n)(*[p._h for p in plans])
        e = C.c_double()
        out = np.zeros(sum(p.n_terms for p in plans), np.float64) if per_term else None
        _check(_lib.mps_expect_pauli_sums(self._h, n, arr, PREC[prec], C.byref(e), _ptr(out)))
        return (e.value, out) if per_term else e.value

    def to_statevector(self) -> np.ndarray:
        """2^N amplitudes, qubit 0 the most significant bit (N <= 26)."""
        psi = np.zeros(1 << self.n, np.complex128)
        _check(_lib.mps_to_statevector(self._h, _ptr(psi.view(np.float64))))
        return psi

    # -- instrumentation ----------------------------------------------------
    def set_fused_gates(self, on: bool = True):
        """Allow or forbid the fused single-gate path of apply_gates."""
        _check(_lib.mps_set_fused_gates(self._h, 1 if on else 0))

    def set_jacobi_groups(self, groups: int = 2):
        """Streams (1..3) over which the batched gate SVD rounds are split."""
        _check(_lib.mps_set_jacobi_groups(self._h, int(groups)))

    def set_autotune(self, on: bool = True):
        """Choose the environment GEMM tile shapes by measurement (c128, c64)."""
        _check(_lib.mps_set_autotune(self._h, 1 if on else 0))

    def copy_from(self, src: "Mps"):
        """Take src's state (same qubit count and bond capacities)."""
        _check(_lib.mps_copy(self._h, src._h))

    def set_graphs(self, on: bool = True):
        """Replay the expectation's device work as a captured HIP graph."""
        _check(_lib.mps_set_graphs(self._h, 1 if on else 0))

    def set_env_tile(self, tile: int = -1):
        """Force one environment GEMM tile shape (0..7); -1 restores the default."""
        _check(_lib.mps_set_env_tile(self._h, int(tile)))

    def set_timing(self, on: bool = True):
        _check(_lib.mps_set_timing(self._h, 1 if on else 0))

    def timing(self) -> dict:
        t = Timing()
        _check(_lib.mps_get_timing(self._h, C.byref(t)))
        return t.as_dict()

    def device_bytes(self) -> int:
        v = C.c_size_t()
        _check(_lib.mps_device_bytes(self._h, C.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.mps_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def apply_gates_multi(mpss, gate_lists, stream=None) -> np.ndarray:
    """Apply gate_lists[i] = (q0, q1, u_packed) to mpss[i] for every i in one
    sequence of device launches (the gate chains advance together, one
    workgroup per MPS).  Returns the number of gates applied per MPS; on a
    failed gate raises MpsError with .n_done set to that array."""
    n = len(mpss)
    if n != len(gate_lists):
        raise ValueError("one gate list per MPS")
    keep = []
    hs = (C.c_void_p * n)()
    p0 = (C.c_void_p * n)()
    p1 = (C.c_void_p * n)()
    pu = (C.c_void_p * n)()
    ng = np.zeros(n, np.int64)
    for i, (m, (q0, q1, u)) in enumerate(zip(mpss, gate_lists)):
        q0 = np.ascontiguousarray(q0, dtype=np.int32)
        q1 = np.ascontiguousarray(q1, dtype=np.int32)
        u = np.ascontiguousarray(u, dtype=np.float64)
        if q1.size != q0.size or u.size != 32 * q0.size:
            raise ValueError("u_packed must hold 32 doubles per gate")
        keep += [q0, q1, u]
        hs[i] = m._h
        p0[i], p1[i], pu[i] = _ptr(q0), _ptr(q1), _ptr(u)
        ng[i] = q0.size
    done = np.zeros(n, np.int64)
    try:
        _check(_lib.mps_apply_gates_multi(n, C.cast(hs, C.c_void_p), _ptr(ng), C.cast(p0, C.c_void_p),
                                          C.cast(p1, C.c_void_p), C.cast(pu, C.c_void_p),
                                          stream, _ptr(done)))
    except MpsError as err:
        err.n_done = done
        raise
    return done


def expect_multi(states, plans, prec: str = "c128", per_term: bool = False):
    """E of every (state, plan) pair in one pass: environment launches of equal
    depth are shared by all states.  Returns an array of energies (and the
    per-string values of each plan)."""
    n = len(states)
    if len(plans) != n:
        raise ValueError("one plan per state")
    lib = load()
    hs = (C.c_void_p * n)(*[m._h for m in states])
    ps = (C.c_void_p * n)(*[p._h for p in plans])
    e = np.zeros(n, np.float64)
    outs = [np.zeros(p.n_terms, np.float64) for p in plans] if per_term else None
    pt = (C.c_void_p * n)(*[o.ctypes.data for o in outs]) if per_term else None
    _check(lib.mps_expect_pauli_sum_multi(n, hs, ps, PREC[prec], _ptr(e), pt))
    return (e, outs) if per_term else e


def jacobi_svd(vectors: np.ndarray):
    """Algorithm 1 on the rows of `vectors` (n_vec x len): returns (sigma, W, sweeps)
    with vectors = U diag(sigma) W."""
    lib = load()
    v = _cplx(vectors)
    n, m = v.shape
    sig = np.zeros(n, np.float64)
    out = np.zeros((n, m), np.complex128)
    sw = C.c_int32()
    _check(lib.mps_jacobi_svd(n, m, _ptr(v.view(np.float64)), _ptr(sig),
                              _ptr(out.view(np.float64)), C.byref(sw)))
    return sig, out, sw.value


def jacobi_svd_noalloc(vectors: np.ndarray, stream: int | None = None):
    """As jacobi_svd, through the entry point that allocates no device memory
    (fixed per-device scratch; at most 512 vectors of at most 512 elements)."""
    lib = load()
    v = _cplx(vectors)
    n, m = v.shape
    sig = np.zeros(n, np.float64)
    out = np.zeros((n, m), np.complex128)
    sw = C.c_int32()
    _check(lib.mps_jacobi_svd_noalloc(n, m, _ptr(v.view(np.float64)), _ptr(sig),
                                      _ptr(out.view(np.float64)), C.byref(sw), stream))
    return sig, out, sw.value


def selftest_mfma() -> np.ndarray:
    """(4, 16, 16): the FP64 and FP32 16x16x4 and the bf16 and f16 16x16x32
    products of the layout check."""
    lib = load()
    out = np.zeros((4, 16, 16), np.float64)
    _check(lib.mps_selftest_mfma(_ptr(out)))
    return out


def autotune_table() -> list[dict]:
    """Tuned launch classes: device, precision, GEMM half, D_l, D_r, item
    bucket, the chosen tile index and shape, and the time of every tile."""
    lib = load()
    n = C.c_int64(0)
    _check(lib.mps_autotune_table(None, 0, C.byref(n)))
    buf = C.create_string_buffer(max(n.value, 1))
    _check(lib.mps_autotune_table(buf, n.value, C.byref(n)))
    rows = []
    for line in buf.value.decode().splitlines():
        f = line.split()
        rows.append({"device": int(f[0]), "prec": f[1], "half": int(f[2]), "dl": int(f[3]),
                     "dr": int(f[4]), "bucket": int(f[5]), "tile": int(f[6]), "shape": f[7],
                     "ms": [float(x) for x in f[8:]]})
    return rows


def autotune_reset():
    _check(load().mps_autotune_reset())
