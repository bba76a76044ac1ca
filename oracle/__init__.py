"""CPU oracle for the codon-constrained McCaskill partition function.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
path (the HIP library and its binding) never touches it.

``liboracle.so`` is built from ``oracle.c`` (codon-state dynamic program,
reverse-mode marginals, exact sampler) and ``seqmcc.c`` (single-sequence
McCaskill used as a pin) with gcc; ``brute.py`` enumerates sequences and
structures directly.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["oracle.c", "seqmcc.c", "mfe.c", "tensor.c"]
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (OpenMP over the cells of a diagonal)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", _LIB_PATH]
        cmd += [os.path.join(_HERE, s) for s in _SOURCES] + ["-lm"]
        subprocess.run(cmd, check=True)
    return _LIB_PATH


def build_variant(out_path: str, defines) -> str:
    """Build a throwaway copy of the oracle with extra -D switches (the
    planted-mistake variants used by tests/test_oracle_mutations.py)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", out_path]
    cmd += ["-D" + d for d in defines]
    cmd += [os.path.join(_HERE, s) for s in _SOURCES] + ["-lm"]
    subprocess.run(cmd, check=True)
    return out_path


def load(path: str):
    """Open an oracle library and declare its entry points."""
    return _configure(ctypes.CDLL(path))


def use(L) -> None:
    """Route this module's functions to library L (None: the default build)."""
    global _lib
    _lib = L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _configure(ctypes.CDLL(_LIB_PATH))
    return _lib


def _configure(L):
    if True:
        d = ctypes.POINTER(ctypes.c_double)
        L.orc_logz.argtypes = [ctypes.c_int, ctypes.c_char_p, d, d, d, d]
        L.orc_logz.restype = ctypes.c_int
        L.orc_marginals.argtypes = [ctypes.c_int, ctypes.c_char_p, d, d, d, d, d, d, d, d, d, d]
        L.orc_marginals.restype = ctypes.c_int
        L.orc_slot_base.argtypes = [ctypes.c_char, ctypes.c_int, ctypes.c_int]
        L.orc_slot_base.restype = ctypes.c_int
        L.orc_num_threads.restype = ctypes.c_int
        ip = ctypes.POINTER(ctypes.c_int)
        L.seq_logz.argtypes = [ctypes.c_int, ip, d, ctypes.c_int, ctypes.c_int]
        L.seq_logz.restype = ctypes.c_double
        L.seq_energy_eval.argtypes = [ctypes.c_int, ip, ip, d]
        L.seq_energy_eval.restype = ctypes.c_double
        if hasattr(L, "orc_sample"):
            L.orc_sample.argtypes = [ctypes.c_int, ctypes.c_char_p, d, d, d, ctypes.c_uint64,
                                     ctypes.c_int, ctypes.POINTER(ctypes.c_uint8),
                                     ctypes.POINTER(ctypes.c_int32)]
            L.orc_sample.restype = ctypes.c_int
        if hasattr(L, "orc_mfe"):
            L.orc_mfe.argtypes = [ctypes.c_int, ctypes.c_char_p, d, d, d, d, ctypes.POINTER(ctypes.c_uint8),
                                  ctypes.POINTER(ctypes.c_int32)]
            L.orc_mfe.restype = ctypes.c_int
        if hasattr(L, "orc_tensor_logz"):
            L.orc_tensor_logz.argtypes = [ctypes.c_int, ctypes.c_char_p, d, ctypes.c_int, ctypes.c_int, d, d, d, d, d]
            L.orc_tensor_logz.restype = ctypes.c_int
            L.orc_tensor_dims.argtypes = [ctypes.c_int, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)]
            L.orc_tensor_dims.restype = ctypes.c_int
        if hasattr(L, "orc_subopt"):
            L.orc_subopt.argtypes = [ctypes.c_int, ctypes.c_char_p, d, d, d, ctypes.c_double, ctypes.c_int, d, d,
                                     ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int)]
            L.orc_subopt.restype = ctypes.c_int
        if hasattr(L, "orc_philox_u01"):
            L.orc_philox_u01.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
            L.orc_philox_u01.restype = ctypes.c_double
    return L


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _prep(prob):
    m = len(prob.prot)
    t1 = None if prob.theta1 is None else np.ascontiguousarray(prob.theta1, dtype=np.float64)
    t2 = None if prob.theta2 is None else np.ascontiguousarray(prob.theta2, dtype=np.float64)
    return m, prob.prot.encode(), t1, t2


def logz(prob, energy) -> float:
    m, aa, t1, t2 = _prep(prob)
    en = energy.packed()
    out = np.zeros(1)
    rc = lib().orc_logz(m, aa, _dp(t1), _dp(t2), _dp(en), _dp(out))
    if rc != 0:
        raise RuntimeError(f"oracle orc_logz failed ({rc})")
    return float(out[0])


def marginals(prob, energy, checks: bool = False) -> dict:
    """log Z, pair [n,n], base [n,4], codon [m,6], codon_pair [m,6,6]."""
    m, aa, t1, t2 = _prep(prob)
    n = 3 * m
    en = energy.packed()
    out = {
        "logz": np.zeros(1), "pair": np.zeros((n, n)), "base": np.zeros((n, 4)),
        "codon": np.zeros((m, 6)), "codon_pair": np.zeros((m, 6, 6)),
    }
    vchk = np.zeros(n) if checks else None
    echk = np.zeros(max(n - 1, 1)) if checks else None
    rc = lib().orc_marginals(m, aa, _dp(t1), _dp(t2), _dp(en), _dp(out["logz"]),
                             _dp(out["pair"]), _dp(out["base"]), _dp(out["codon"]),
                             _dp(out["codon_pair"]), _dp(vchk), _dp(echk))
    if rc != 0:
        raise RuntimeError(f"oracle orc_marginals failed ({rc})")
    out["logz"] = float(out["logz"][0])
    if checks:
        out["vcheck"] = vchk
        out["echeck"] = echk[: n - 1]
    return out


def sample(prob, energy, seed: int, nsamp: int):
    """Exact joint samples: codon slots [N, m] (uint8) and pair tables [N, n]."""
    m, aa, t1, t2 = _prep(prob)
    n = 3 * m
    en = energy.packed()
    cod = np.zeros((nsamp, m), dtype=np.uint8)
    pairs = np.zeros((nsamp, n), dtype=np.int32)
    rc = lib().orc_sample(m, aa, _dp(t1), _dp(t2), _dp(en), ctypes.c_uint64(seed), nsamp,
                          cod.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                          pairs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc != 0:
        raise RuntimeError(f"oracle orc_sample failed ({rc})")
    return cod, pairs


def mfe(prob, energy, traceback: bool = True):
    """Minimum free energy (kT) over codon sequences and structures
    (mfe.c), and one minimising state: codon slots [m] (uint8) and the pair
    table [n] (-1 unpaired), or (mfe, None, None)."""
    m, aa, t1, t2 = _prep(prob)
    en = energy.packed()
    out = np.zeros(1)
    cod = np.zeros(m, np.uint8) if traceback else None
    pairs = np.zeros(3 * m, np.int32) if traceback else None
    rc = lib().orc_mfe(m, aa, _dp(t1), _dp(t2), _dp(en), _dp(out),
                       None if cod is None else cod.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                       None if pairs is None else pairs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc != 0:
        raise RuntimeError(f"oracle orc_mfe failed ({rc})")
    return float(out[0]), cod, pairs


def subopt(prob, energy, gap: float, max_states: int = 10000):
    """Every state within gap (kT) of the MFE (mfe.c, depth-first order):
    (mfe, energies [k], codons [k, m] uint8, pairs [k, n] int32, complete),
    complete False when more than max_states states exist."""
    m, aa, t1, t2 = _prep(prob)
    en = energy.packed()
    out = np.zeros(1)
    energies = np.zeros(max(max_states, 1))
    cod = np.zeros((max(max_states, 1), m), np.uint8)
    pairs = np.zeros((max(max_states, 1), 3 * m), np.int32)
    cnt = ctypes.c_int(0)
    rc = lib().orc_subopt(m, aa, _dp(t1), _dp(t2), _dp(en), float(gap), int(max_states), _dp(out), _dp(energies),
                          cod.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                          pairs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(cnt))
    if rc < 0:
        raise RuntimeError(f"oracle orc_subopt failed ({rc})")
    k = cnt.value
    return float(out[0]), energies[:k].copy(), cod[:k].copy(), pairs[:k].copy(), rc == 0


def tensor_logz(prob, model):
    """log Z of the tensor-based model summed over the protein's codon
    sequences (tensor.c) and the prefix values log Z(first a residues),
    a = 1..m.  Codon bonuses theta1 (if any) weight the middle cores."""
    m, aa, t1, _ = _prep(prob)
    V = np.ascontiguousarray(model.V, np.float64)
    B = np.ascontiguousarray(model.B, np.float64)
    S = np.ascontiguousarray(model.S, np.float64)
    out = np.zeros(1)
    pre = np.zeros(m)
    rc = lib().orc_tensor_logz(m, aa, _dp(t1), model.gamma, model.xi, _dp(V), _dp(B), _dp(S), _dp(out), _dp(pre))
    if rc != 0:
        raise RuntimeError(f"oracle orc_tensor_logz failed ({rc})")
    return float(out[0]), pre


def tensor_dims(prot: str) -> np.ndarray:
    """Bond dimensions Sigma_p, p = 0..n, of the single-codon tensor train."""
    sig = np.zeros(3 * len(prot) + 1, np.int32)
    rc = lib().orc_tensor_dims(len(prot), prot.encode(), sig.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if rc != 0:
        raise RuntimeError(f"oracle orc_tensor_dims failed ({rc})")
    return sig


def philox_u01(seed: int, sample_id: int, draw: int) -> float:
    return lib().orc_philox_u01(ctypes.c_uint64(seed), sample_id, draw)


def slot_base(aa: str, s: int, r: int) -> int:
    return lib().orc_slot_base(aa.encode(), s, r)


def seq_logz(seq, energy, forbid=None) -> float:
    s = np.ascontiguousarray(seq, dtype=np.int32)
    en = energy.packed()
    fi, fj = forbid if forbid is not None else (-1, -1)
    return lib().seq_logz(len(s), s.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(en), fi, fj)


def seq_energy(seq, pt, energy) -> float:
    s = np.ascontiguousarray(seq, dtype=np.int32)
    p = np.ascontiguousarray(pt, dtype=np.int32)
    en = energy.packed()
    return lib().seq_energy_eval(len(s), s.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                 p.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(en))


def num_threads() -> int:
    return lib().orc_num_threads()
