"""Oracle for frequency matching (Section S4e, algorithm "iterative").

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by tests and
by nothing on the product path.

Codon bonuses f (one positive number per codon; a codon is a residue letter
and one of its slots) enter the model as position log weights
theta1[a][s] = log f(letter of residue a, s).  The target frequencies b* are
those of independent codon choice with the target bonuses f*: each residue
of letter L takes slot s with probability f*(L, s) / sum_t f*(L, t), so
b*(L, s) = count(L) * f*(L, s) / sum_t f*(L, t).  The achieved frequencies
b(L, s) are the codon marginals (Section 2c, eq. codon-marginal) summed over
the residues of letter L.

The fixed-point map acts on x = log f:
    r(x) = log b* - log b(x),    g(x) = x + r(x),
which is the prose's update (multiply the bonuses by desired over achieved
frequencies).  The printed algorithm multiplies by achieved over desired; that
moves away from the target (a codon sampled too often would gain weight), so
the prose is taken as the definition.  Iteration stops when
max |log(b / b*)| < r_tol over the codons present in the protein.

Anderson acceleration (Walker and Ni, SIAM J. Numer. Anal. 49 (2011),
Algorithm AA with unit mixing): with history m_k = min(m, k),
    DR = [r_{k-m_k+1} - r_{k-m_k}, ..., r_k - r_{k-1}],  DG likewise for g,
    gamma = argmin || r_k - DR gamma ||_2,
    x_{k+1} = g_k - DG gamma.
m = 0 is the plain fixed-point iteration; m < 0 keeps the whole history (the
paper's runs had no history limit); m_k never exceeds the dimension of x.
"""
from __future__ import annotations

from typing import Callable, Optional

import numpy as np

from . import lib, marginals

NLET = 26   # rows of a bonus table: residue letter - 'A'
NSLOT = 6


def degeneracy(letter: str) -> int:
    """Number of codons of a residue letter, from this oracle's genetic code."""
    d = 0
    while d < NSLOT and lib().orc_slot_base(letter.encode(), d, 0) >= 0:
        d += 1
    return d


def present_mask(prot: str) -> np.ndarray:
    """[26][6] bool: codons (letter, slot) of the letters present in prot."""
    mask = np.zeros((NLET, NSLOT), dtype=bool)
    for L in set(prot):
        mask[ord(L) - 65, :degeneracy(L)] = True
    return mask


def target_frequencies(prot: str, f_target: np.ndarray) -> np.ndarray:
    """b*: expected codon counts of independent codon choice with bonuses f_target."""
    b = np.zeros((NLET, NSLOT))
    for L in set(prot):
        r, d = ord(L) - 65, degeneracy(L)
        w = np.asarray(f_target[r, :d], dtype=np.float64)
        b[r, :d] = prot.count(L) * w / w.sum()
    return b


def achieved_frequencies(prot: str, codon: np.ndarray) -> np.ndarray:
    """b: codon marginals [m][6] summed over the residues of each letter."""
    b = np.zeros((NLET, NSLOT))
    for a, L in enumerate(prot):
        d = degeneracy(L)
        b[ord(L) - 65, :d] += codon[a, :d]
    return b


def theta1_of(prot: str, x: np.ndarray) -> np.ndarray:
    """Position log weights theta1[a][s] = x(letter of a, s)."""
    t = np.zeros((len(prot), NSLOT))
    for a, L in enumerate(prot):
        d = degeneracy(L)
        t[a, :d] = x[ord(L) - 65, :d]
    return t


def anderson(g: Callable[[np.ndarray], np.ndarray], x0: np.ndarray, tol: float, max_eval: int,
             history: int = -1, norm=lambda r: float(np.max(np.abs(r)))):
    """Fixed point of g by Anderson acceleration (Walker and Ni, Algorithm AA,
    unit mixing) on flat vectors.  Returns (x, errors, converged): errors[k] is
    norm(g(x_k) - x_k) of evaluation k; x is the iterate whose residual met tol
    (else the last one evaluated)."""
    x = np.array(x0, dtype=np.float64)
    xs, rs, gs, errs = [], [], [], []
    for k in range(max_eval):
        gx = g(x)
        r = gx - x
        errs.append(norm(r))
        if errs[-1] < tol:
            return x, errs, True
        xs.append(x)
        rs.append(r)
        gs.append(gx)
        mk = k if history < 0 else min(history, k)
        mk = min(mk, x.size)  # no more differences than dimensions
        if mk == 0:
            x = gx
            continue
        DR = np.stack([rs[i + 1] - rs[i] for i in range(k - mk, k)], axis=1)
        DG = np.stack([gs[i + 1] - gs[i] for i in range(k - mk, k)], axis=1)
        gamma = np.linalg.lstsq(DR, r, rcond=None)[0]
        x = gx - DG @ gamma
    return xs[-1], errs, False


def match_frequencies(prob, energy, f_target: np.ndarray, r_tol: float = 0.002,
                      max_eval: int = 30, history: int = -1,
                      marg: Optional[Callable] = None):
    """Codon bonuses whose Boltzmann codon frequencies match b* of f_target.

    prob: .prot, .theta2 (theta1 is replaced by log f).  f_target [26][6] > 0 on
    the codons of the protein.  Returns (f [26][6], errors per evaluation,
    converged).  marg(prob, energy) -> codon marginals [m][6] defaults to this
    oracle's marginals."""
    prot = prob.prot
    mask = present_mask(prot)
    bstar = target_frequencies(prot, f_target)
    lbs = np.log(bstar[mask])

    class _P:
        pass

    def codon_marginals(x_full):
        p = _P()
        p.prot, p.theta1, p.theta2 = prot, theta1_of(prot, x_full), prob.theta2
        if marg is not None:
            return marg(p, energy)
        return marginals(p, energy)["codon"]

    def g(xa):
        x_full = np.zeros((NLET, NSLOT))
        x_full[mask] = xa
        b = achieved_frequencies(prot, codon_marginals(x_full))
        return xa + (lbs - np.log(b[mask]))

    x0 = np.log(np.asarray(f_target, dtype=np.float64)[mask])
    xa, errs, ok = anderson(g, x0, r_tol, max_eval, history)
    f = np.zeros((NLET, NSLOT))
    f[mask] = np.exp(xa)
    return f, errs, ok
