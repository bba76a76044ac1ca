"""Brute-force enumeration of the joint ensemble (test infrastructure only).

Sums W(c) * exp(-E(phi(c), s)) over EVERY codon assignment c and EVERY
non-crossing structure s of phi(c), straight from the definitions of the
paper's Section 2b (eqs. structure-q, sequence-q, amino-q with the bias of the
soft constraints) and the marginals of Section 2c (eqs. pair-probability,
marginal-base, marginal-codon).  The loop energy E is evaluated here by a
plain loop decomposition of each structure, written independently of both C
files.  Feasible for proteins of a few residues only.
"""
from __future__ import annotations

import itertools
import math
from functools import lru_cache

import numpy as np

BASES = "ACGU"
PAIR_TYPES = {("A", "U"): 0, ("C", "G"): 1, ("G", "C"): 2, ("U", "A"): 3,
              ("G", "U"): 4, ("U", "G"): 5}


def load_genetic_code(path: str) -> dict:
    """aa -> codons in canonical slot order (lexicographic in A<C<G<U)."""
    code = {}
    with open(path) as f:
        for ln in f:
            ln = ln.strip()
            if not ln or ln.startswith("#"):
                continue
            parts = ln.split()
            if parts[0] == ">":
                continue
            code[parts[0]] = sorted(parts[1:], key=lambda c: [BASES.index(x) for x in c])
    return code


def structures(seq: str):
    """All non-crossing structures (tuples of pairs) with canonical pairs and
    hairpins of at least 3 unpaired bases."""
    n = len(seq)

    @lru_cache(maxsize=None)
    def rec(i, j):
        if i > j:
            return [()]
        out = list(rec(i + 1, j))  # i unpaired
        for k in range(i + 4, j + 1):
            if (seq[i], seq[k]) in PAIR_TYPES:
                for inner in rec(i + 1, k - 1):
                    for rest in rec(k + 1, j):
                        out.append(((i, k),) + inner + rest)
        return out

    return rec(0, n - 1)


def loop_energy(seq: str, pairs, E) -> float:
    """Free energy (kT) of one structure as a sum over its loops."""
    n = len(seq)
    pt = [-1] * n
    for i, j in pairs:
        pt[i], pt[j] = j, i
    total = 0.0
    for i, j in pairs:
        t = PAIR_TYPES[(seq[i], seq[j])]
        children, unpaired = [], 0
        k = i + 1
        while k < j:
            if pt[k] > k:
                children.append((k, pt[k]))
                k = pt[k] + 1
            else:
                unpaired += 1
                k += 1
        b = lambda x: BASES.index(x)
        if not children:
            L = j - i - 1
            h = E.hairpin[L] if L <= 30 else E.hairpin[30] + E.extrap * math.log(L / 30.0)
            total += h + E.mismatch[b(seq[i + 1])][b(seq[j - 1])][t]
        elif len(children) == 1:
            k, l = children[0]
            l1, l2 = k - i - 1, j - l - 1
            if l1 + l2 > 30:
                return math.inf
            if l1 == 0 and l2 == 0:
                total += E.stack[t][PAIR_TYPES[(seq[k], seq[l])]]
            elif l1 == 0 or l2 == 0:
                total += E.bulge[l1 + l2]
            else:
                total += (E.interior[l1 + l2] + E.mismatch[b(seq[i + 1])][b(seq[j - 1])][t]
                          + E.mismatch[b(seq[l + 1])][b(seq[k - 1])][PAIR_TYPES[(seq[l], seq[k])]])
        else:
            total += E.ml_a + E.ml_b * (len(children) + 1) + E.ml_c * unpaired
    return total


def log_weight(prob, c) -> float:
    """log W(c): codon weights plus codon-pair weights across boundaries."""
    w = 0.0
    for a, s in enumerate(c):
        if prob.theta1 is not None:
            w += prob.theta1[a][s]
        if a >= 1 and prob.theta2 is not None:
            w += prob.theta2[a][c[a - 1]][s]
    return w


def enumerate_ensemble(prob, E, code: dict):
    """Exact log Z and marginals; also Pr(c) for every codon assignment and the
    list of (c, structure, probability) states."""
    prot = prob.prot
    m, n = len(prot), 3 * len(prot)
    slots = [range(len(code[ch])) for ch in prot]
    states = []
    for c in itertools.product(*slots):
        seq = "".join(code[ch][s] for ch, s in zip(prot, c))
        lw = log_weight(prob, c)
        for st in structures(seq):
            e = loop_energy(seq, st, E)
            if math.isfinite(e):
                states.append((c, st, lw - e, seq))
    mx = max(s[2] for s in states)
    ws = np.array([math.exp(s[2] - mx) for s in states])
    Z = ws.sum()
    logz = math.log(Z) + mx
    p = ws / Z
    pair = np.zeros((n, n))
    codon = np.zeros((m, 6))
    cpair = np.zeros((m, 6, 6))
    base = np.zeros((n, 4))
    seqprob = {}
    for (c, st, _, seq), pr in zip(states, p):
        for i, j in st:
            pair[i, j] += pr
            pair[j, i] += pr
        for a, s in enumerate(c):
            codon[a, s] += pr
            if a >= 1:
                cpair[a, c[a - 1], s] += pr
        for k, ch in enumerate(seq):
            base[k, BASES.index(ch)] += pr
        seqprob[c] = seqprob.get(c, 0.0) + pr
    for i in range(n):
        pair[i, i] = 1.0 - pair[i].sum()
    joint = [(c, st, pr) for (c, st, _, _), pr in zip(states, p)]
    return {"logz": logz, "pair": pair, "codon": codon, "codon_pair": cpair,
            "base": base, "seqprob": seqprob, "joint": joint, "count": len(states)}


def count_structures(prob, code: dict) -> int:
    """Sum over sequences of the number of structures (all energies zero)."""
    tot = 0
    for c in itertools.product(*[range(len(code[ch])) for ch in prob.prot]):
        seq = "".join(code[ch][s] for ch, s in zip(prob.prot, c))
        tot += len(structures(seq))
    return tot
