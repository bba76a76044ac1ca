"""ctypes binding of libcdz.so: argument marshalling only.

Every function here has the name of the C entry point it calls and does no
arithmetic of its own; all dynamic programming runs in the HIP library.  The
binding raises if the library is not built (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcdz.so")

CDZ_FP32_SCALED = 0
CDZ_FP64 = 1
ENERGY_LEN = 229  # doubles in the cdz_energy record
STATUS = ["CDZ_OK", "CDZ_ERR_ARG", "CDZ_ERR_PROTEIN", "CDZ_ERR_NUMERIC", "CDZ_ERR_NOMEM",
          "CDZ_ERR_BUDGET", "CDZ_ERR_HIP", "CDZ_ERR_STATE"]
EXPORTS = ["cdz_create", "cdz_destroy", "cdz_partition", "cdz_marginals", "cdz_sample", "cdz_sample_noalloc",
           "cdz_forward_dev", "cdz_backward_dev", "cdz_last_timings", "cdz_reset",
           "cdz_set_profiling", "cdz_kernel_timings", "cdz_status_string", "cdz_last_error",
           "cdz_batch", "cdz_partition_batch", "cdz_marginals_batch", "cdz_sample_batch",
           "cdz_workspace_bytes", "cdz_match_frequencies", "cdz_mfe", "cdz_subopt", "cdz_tensor_logz",
           "cdz_tensor_dims"]

_dp = ctypes.POINTER(ctypes.c_double)


class cdz_problem(ctypes.Structure):
    _fields_ = [("n_aa", ctypes.c_int32), ("aa", ctypes.c_char_p),
                ("theta1", _dp), ("theta2", _dp)]


class cdz_options(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("mem_budget_bytes", ctypes.c_size_t),
                ("hip_stream", ctypes.c_void_p)]


class cdz_tensor_model(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_int32), ("xi", ctypes.c_int32), ("V", _dp), ("B", _dp), ("S", _dp)]


class CdzError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS[status] if 0 <= status < len(STATUS) else status}: {msg}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        # PyTorch ships its own HIP runtime under the same soname as the system
        # one the library links; whichever is loaded first serves the whole
        # process, and torch cannot start its device on a runtime other than
        # its own.  Load torch's first so that one runtime serves both.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        sig = {
            "cdz_create": ([_dp, ctypes.POINTER(cdz_options), ctypes.POINTER(vp)], ctypes.c_int),
            "cdz_destroy": ([vp], None),
            "cdz_partition": ([vp, ctypes.POINTER(cdz_problem), _dp], ctypes.c_int),
            "cdz_marginals": ([vp, ctypes.POINTER(cdz_problem), _dp, _dp, _dp, _dp, _dp], ctypes.c_int),
            "cdz_sample": ([vp, ctypes.POINTER(cdz_problem), ctypes.c_uint64, ctypes.c_int32,
                            ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "cdz_sample_noalloc": ([vp, ctypes.POINTER(cdz_problem), ctypes.c_uint64, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "cdz_forward_dev": ([vp, ctypes.c_int32, ctypes.c_char_p, vp, vp, _dp], ctypes.c_int),
            "cdz_backward_dev": ([vp, ctypes.c_double, vp, vp], ctypes.c_int),
            "cdz_last_timings": ([vp, _dp], ctypes.c_int),
            "cdz_status_string": ([ctypes.c_int], ctypes.c_char_p),
            "cdz_last_error": ([vp], ctypes.c_char_p),
            "cdz_debug_logz_suffix": ([vp], ctypes.c_double),
            "cdz_reset": ([vp], ctypes.c_int),
            "cdz_set_profiling": ([vp, ctypes.c_int], ctypes.c_int),
            "cdz_kernel_timings": ([vp, _dp], ctypes.c_int),
            "cdz_batch": ([vp, ctypes.POINTER(cdz_problem), ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                           _dp, _dp, _dp, _dp, _dp, ctypes.POINTER(ctypes.c_uint8),
                           ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "cdz_partition_batch": ([vp, ctypes.POINTER(cdz_problem), ctypes.c_int32, _dp], ctypes.c_int),
            "cdz_marginals_batch": ([vp, ctypes.POINTER(cdz_problem), ctypes.c_int32, _dp, _dp, _dp, _dp,
                                     _dp], ctypes.c_int),
            "cdz_sample_batch": ([vp, ctypes.POINTER(cdz_problem), ctypes.c_int32, ctypes.c_uint64,
                                  ctypes.c_int32, ctypes.POINTER(ctypes.c_uint8),
                                  ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "cdz_workspace_bytes": ([vp, ctypes.POINTER(cdz_problem), ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
            "cdz_tensor_logz": ([vp, ctypes.POINTER(cdz_tensor_model), ctypes.POINTER(cdz_problem), _dp, _dp],
                                ctypes.c_int),
            "cdz_tensor_dims": ([ctypes.POINTER(cdz_problem), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "cdz_subopt": ([vp, ctypes.POINTER(cdz_problem), ctypes.c_double, ctypes.c_int32, _dp, _dp,
                            ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32),
                            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "cdz_mfe": ([vp, ctypes.POINTER(cdz_problem), _dp, ctypes.POINTER(ctypes.c_uint8),
                         ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "cdz_match_frequencies": ([vp, ctypes.POINTER(cdz_problem), _dp, ctypes.c_double, ctypes.c_int32,
                                       ctypes.c_int32, _dp, _dp, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            # test hooks of include/cdz_debug.h
            "cdz_debug_al_k": ([vp], ctypes.c_int),
            "cdz_debug_force_al_k": ([vp, ctypes.c_int], ctypes.c_int),
            "cdz_debug_set_span": ([vp, ctypes.c_int], ctypes.c_int),
            "cdz_debug_landscape_retries": ([vp], ctypes.c_int),
            "cdz_debug_set_low_exp": ([vp, ctypes.c_int], ctypes.c_int),
            "cdz_debug_set_graphs": ([vp, ctypes.c_int], ctypes.c_int),
            "cdz_debug_set_fuse": ([vp, ctypes.c_int], ctypes.c_int),
            "cdz_debug_graph_counts": ([vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
                                       ctypes.c_int),
            "cdz_debug_weakest": ([vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
            "cdz_debug_copy": ([vp, ctypes.c_int, vp, ctypes.c_size_t,
                                ctypes.POINTER(ctypes.c_longlong)], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.argtypes = args
                f.restype = res
        _lib = L
    return _lib


def _arr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_dp)


class _Prob:
    """Keeps the marshalled buffers alive while a call runs."""

    def __init__(self, prob):
        self.aa = prob.prot.encode()
        self.t1 = None if prob.theta1 is None else np.ascontiguousarray(prob.theta1, np.float64)
        self.t2 = None if prob.theta2 is None else np.ascontiguousarray(prob.theta2, np.float64)
        self.c = cdz_problem(len(prob.prot), self.aa, _arr(self.t1), _arr(self.t2))


class Handle:
    def __init__(self, ptr, energy_buf):
        self.ptr = ptr
        self._energy = energy_buf

    def __del__(self):
        try:
            if self.ptr:
                lib().cdz_destroy(self.ptr)
        except Exception:
            pass
        self.ptr = None

    def check(self, st: int):
        if st != 0:
            msg = lib().cdz_last_error(self.ptr).decode(errors="replace")
            raise CdzError(st, msg)


def cdz_create(energy, prec: str = "fp32", mem_budget_bytes: int = 0, stream: int = 0) -> Handle:
    """energy: an object with .packed() (229 doubles in cdz_energy order)."""
    buf = np.ascontiguousarray(energy.packed(), np.float64)
    if buf.shape != (ENERGY_LEN,):
        raise ValueError(f"energy record must be {ENERGY_LEN} doubles, got shape {buf.shape}")
    opts = cdz_options(CDZ_FP64 if prec == "fp64" else CDZ_FP32_SCALED, mem_budget_bytes,
                       ctypes.c_void_p(stream) if stream else None)
    out = ctypes.c_void_p()
    st = lib().cdz_create(_arr(buf), ctypes.byref(opts), ctypes.byref(out))
    if st != 0:
        raise CdzError(st, "cdz_create")
    return Handle(out, buf)


def cdz_partition(h: Handle, prob) -> float:
    p = _Prob(prob)
    out = np.zeros(1)
    h.check(lib().cdz_partition(h.ptr, ctypes.byref(p.c), _arr(out)))
    return float(out[0])


def cdz_marginals(h: Handle, prob) -> dict:
    p = _Prob(prob)
    m, n = len(prob.prot), 3 * len(prob.prot)
    out = {"logz": np.zeros(1), "pair": np.zeros((n, n)), "base": np.zeros((n, 4)),
           "codon": np.zeros((m, 6)), "codon_pair": np.zeros((m, 6, 6))}
    h.check(lib().cdz_marginals(h.ptr, ctypes.byref(p.c), _arr(out["logz"]), _arr(out["pair"]),
                                _arr(out["base"]), _arr(out["codon"]), _arr(out["codon_pair"])))
    out["logz"] = float(out["logz"][0])
    return out


def cdz_sample(h: Handle, prob, seed: int, n_samples: int):
    p = _Prob(prob)
    m, n = len(prob.prot), 3 * len(prob.prot)
    cod = np.zeros((n_samples, m), np.uint8)
    pairs = np.zeros((n_samples, n), np.int32)
    h.check(lib().cdz_sample(h.ptr, ctypes.byref(p.c), ctypes.c_uint64(seed), n_samples,
                             cod.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                             pairs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return cod, pairs


def cdz_mfe(h: Handle, prob, traceback: bool = True):
    """Minimum free energy (kT) over codon sequences and structures, and one
    minimising state: (mfe, codon slots [n_aa] uint8, pair table [n] int32),
    or (mfe, None, None) without the traceback."""
    p = _Prob(prob)
    m = len(prob.prot)
    out = np.zeros(1)
    cod = np.zeros(m, np.uint8) if traceback else None
    pairs = np.zeros(3 * m, np.int32) if traceback else None
    h.check(lib().cdz_mfe(h.ptr, ctypes.byref(p.c), _arr(out),
                          None if cod is None else cod.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                          None if pairs is None else pairs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return float(out[0]), cod, pairs


def cdz_subopt(h: Handle, prob, gap: float, max_states: int = 10000):
    """Every state within gap (kT) of the minimum free energy: (mfe,
    energies [k], codon slots [k, n_aa] uint8, pair tables [k, n] int32,
    complete), complete False when more than max_states states exist."""
    p = _Prob(prob)
    m, n = len(prob.prot), 3 * len(prob.prot)
    cap = max(int(max_states), 1)
    out = np.zeros(1)
    en = np.zeros(cap)
    cod = np.zeros((cap, m), np.uint8)
    pairs = np.zeros((cap, n), np.int32)
    cnt = ctypes.c_int32(0)
    more = ctypes.c_int32(0)
    h.check(lib().cdz_subopt(h.ptr, ctypes.byref(p.c), float(gap), int(max_states), _arr(out), _arr(en),
                             cod.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                             pairs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(cnt),
                             ctypes.byref(more)))
    k = cnt.value
    return float(out[0]), en[:k].copy(), cod[:k].copy(), pairs[:k].copy(), more.value == 0


def cdz_tensor_logz(h: Handle, model, prob):
    """log Z of prob (theta2 must be None) under a tensor-based model
    (``inputs.TensorModel``) in the handle's precision, and the prefix values
    log Z(first a residues), a = 1..n_aa."""
    p = _Prob(prob)
    V = np.ascontiguousarray(model.V, np.float64)
    Bm = np.ascontiguousarray(model.B, np.float64)
    S = np.ascontiguousarray(model.S, np.float64)
    md = cdz_tensor_model(model.gamma, model.xi, _arr(V), _arr(Bm), _arr(S))
    out = np.zeros(1)
    pre = np.zeros(len(prob.prot))
    h.check(lib().cdz_tensor_logz(h.ptr, ctypes.byref(md), ctypes.byref(p.c), _arr(out), _arr(pre)))
    return float(out[0]), pre


def cdz_tensor_dims(prob) -> np.ndarray:
    """Bond dimensions Sigma_p, p = 0..n, of the protein's single-codon train."""
    p = _Prob(prob)
    sig = np.zeros(3 * len(prob.prot) + 1, np.int32)
    st = lib().cdz_tensor_dims(ctypes.byref(p.c), sig.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if st != 0:
        raise CdzError(st, "cdz_tensor_dims")
    return sig


def cdz_match_frequencies(h: Handle, prob, f_target: np.ndarray, r_tol: float = 0.002,
                          max_eval: int = 30, history: int = -1):
    """Codon bonuses f [26][6] whose ensemble codon frequencies match those of
    independent codon choice with f_target; returns (f, errors per evaluation,
    converged)."""
    p = _Prob(prob)
    ft = np.ascontiguousarray(f_target, dtype=np.float64).reshape(26 * 6)
    f = np.zeros(26 * 6)
    err = np.zeros(max(int(max_eval), 1))
    n_eval = ctypes.c_int32(0)
    conv = ctypes.c_int32(0)
    h.check(lib().cdz_match_frequencies(h.ptr, ctypes.byref(p.c), _arr(ft), float(r_tol), int(max_eval),
                                        int(history), _arr(f), _arr(err), ctypes.byref(n_eval),
                                        ctypes.byref(conv)))
    return f.reshape(26, 6), err[: n_eval.value].copy(), bool(conv.value)


def cdz_sample_noalloc(h: Handle, prob, seed: int, n_samples: int):
    p = _Prob(prob)
    m, n = len(prob.prot), 3 * len(prob.prot)
    cod = np.zeros((n_samples, m), np.uint8)
    pairs = np.zeros((n_samples, n), np.int32)
    h.check(lib().cdz_sample_noalloc(h.ptr, ctypes.byref(p.c), ctypes.c_uint64(seed), n_samples,
                                     cod.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                     pairs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return cod, pairs


class _Batch:
    """Marshalled problem array of a batch and its output offsets."""

    def __init__(self, probs):
        self.items = [_Prob(p) for p in probs]
        self.arr = (cdz_problem * max(1, len(probs)))(*[it.c for it in self.items])
        self.m = [len(p.prot) for p in probs]
        self.n = [3 * x for x in self.m]

    def split(self, flat, sizes, shape):
        out, at = [], 0
        for k, sz in enumerate(sizes):
            out.append(flat[at:at + sz].reshape(shape(k)))
            at += sz
        return out


def cdz_batch(h: Handle, probs, n_samples: int = 0, seed: int = 0, marginals: bool = True) -> dict:
    """One call over a list of problems: log Z of each, marginals (if asked)
    and n_samples samples of each (problem b drawn with seed + b).  Outputs
    are split back into per-problem arrays."""
    B = _Batch(probs)
    cnt = len(probs)
    sn2, sn, sm = sum(x * x for x in B.n), sum(B.n), sum(B.m)
    logz = np.zeros(max(1, cnt))
    pair = np.zeros(sn2) if marginals else None
    base = np.zeros(sn * 4) if marginals else None
    cod1 = np.zeros(sm * 6) if marginals else None
    cod2 = np.zeros(sm * 36) if marginals else None
    sc = np.zeros(max(1, n_samples * sm), np.uint8)
    sp = np.zeros(max(1, n_samples * sn), np.int32)
    h.check(lib().cdz_batch(h.ptr, B.arr, cnt, n_samples, ctypes.c_uint64(seed), _arr(logz), _arr(pair),
                            _arr(base), _arr(cod1), _arr(cod2),
                            sc.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if n_samples else None,
                            sp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if n_samples else None))
    out = {"logz": logz[:cnt].copy()}
    if marginals:
        out["pair"] = B.split(pair, [x * x for x in B.n], lambda k: (B.n[k], B.n[k]))
        out["base"] = B.split(base, [x * 4 for x in B.n], lambda k: (B.n[k], 4))
        out["codon"] = B.split(cod1, [x * 6 for x in B.m], lambda k: (B.m[k], 6))
        out["codon_pair"] = B.split(cod2, [x * 36 for x in B.m], lambda k: (B.m[k], 6, 6))
    if n_samples:
        out["codons"] = B.split(sc, [n_samples * x for x in B.m], lambda k: (n_samples, B.m[k]))
        out["pairs"] = B.split(sp, [n_samples * x for x in B.n], lambda k: (n_samples, B.n[k]))
    return out


CDZ_WS_FORWARD, CDZ_WS_MARGINALS, CDZ_WS_MARGINALS_MIN, CDZ_WS_FORWARD_MIN = 0, 1, 2, 3


def cdz_workspace_bytes(h: Handle, prob, what: int = CDZ_WS_MARGINALS) -> int:
    p = _Prob(prob)
    out = ctypes.c_size_t(0)
    h.check(lib().cdz_workspace_bytes(h.ptr, ctypes.byref(p.c), int(what), ctypes.byref(out)))
    return int(out.value)


def cdz_partition_batch(h: Handle, probs) -> np.ndarray:
    B = _Batch(probs)
    out = np.zeros(max(1, len(probs)))
    h.check(lib().cdz_partition_batch(h.ptr, B.arr, len(probs), _arr(out)))
    return out[:len(probs)].copy()


def cdz_marginals_batch(h: Handle, probs) -> dict:
    return cdz_batch(h, probs, 0, 0, True)


def cdz_sample_batch(h: Handle, probs, seed: int, n_samples: int):
    r = cdz_batch(h, probs, n_samples, seed, False)
    return r.get("codons", []), r.get("pairs", [])


def cdz_forward_dev(h: Handle, aa: str, theta1_ptr: int, theta2_ptr: int) -> float:
    out = np.zeros(1)
    h.check(lib().cdz_forward_dev(h.ptr, len(aa), aa.encode(), ctypes.c_void_p(theta1_ptr),
                                  ctypes.c_void_p(theta2_ptr) if theta2_ptr else None, _arr(out)))
    return float(out[0])


def cdz_backward_dev(h: Handle, grad_logz: float, dtheta1_ptr: int, dtheta2_ptr: int) -> None:
    h.check(lib().cdz_backward_dev(h.ptr, float(grad_logz), ctypes.c_void_p(dtheta1_ptr),
                                   ctypes.c_void_p(dtheta2_ptr) if dtheta2_ptr else None))


def cdz_last_timings(h: Handle) -> np.ndarray:
    out = np.zeros(5)
    h.check(lib().cdz_last_timings(h.ptr, _arr(out)))
    return out


def cdz_reset(h: Handle) -> None:
    h.check(lib().cdz_reset(h.ptr))


def cdz_set_profiling(h: Handle, on: bool) -> None:
    h.check(lib().cdz_set_profiling(h.ptr, 1 if on else 0))


def cdz_kernel_timings(h: Handle) -> np.ndarray:
    out = np.zeros(6)
    h.check(lib().cdz_kernel_timings(h.ptr, _arr(out)))
    return out


def cdz_status_string(st: int) -> str:
    return lib().cdz_status_string(st).decode()


def cdz_last_error(h: Handle) -> str:
    return lib().cdz_last_error(h.ptr).decode(errors="replace")
