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


# ---- tensor-based model (SI S2b, eq. general-model) ------------------------

def all_structures(n: int):
    """All non-crossing structures on n positions whose hairpins have at least
    3 unpaired bases, whatever the bases (the tensor model's B decides which
    pairs carry weight)."""

    @lru_cache(maxsize=None)
    def rec(i, j):
        if i > j:
            return [()]
        out = list(rec(i + 1, j))
        for k in range(i + 4, j + 1):
            for inner in rec(i + 1, k - 1):
                for rest in rec(k + 1, j):
                    out.append(((i, k),) + inner + rest)
        return out

    return rec(0, n - 1)


def tensor_structure_weight(seq: str, pairs, model) -> float:
    """Boltzmann weight of one (sequence, structure) under a tensor model:
    the sum over one rank index per pair of the product over loops of
    Tr[S x (matrices along the loop)] -- V for an unpaired base, B_{x,y} for
    a base x paired to the loop's next base y.  The exterior loop is read
    from the 5' end; a loop closed by (i, j) from the closing pair's 3' side,
    B_{seq[j], seq[i]}, then the bases i+1 .. j-1 at that level."""
    b = [BASES.index(ch) for ch in seq]
    n = len(seq)
    pt = [-1] * n
    for i, j in pairs:
        pt[i], pt[j] = j, i
    g = model.gamma
    total = 0.0
    for rhos in itertools.product(range(model.xi), repeat=len(pairs)):
        rho = {}
        for (i, j), r in zip(pairs, rhos):
            rho[i] = rho[j] = r

        def walk(start, end, M):
            p = start
            while p < end:
                q = pt[p]
                if q < 0:
                    M = M @ model.V[b[p]]
                    p += 1
                else:
                    M = M @ model.B[rho[p], b[p], b[q]]
                    p = q + 1
            return M

        w = np.trace(model.S @ walk(0, n, np.eye(g)))
        for i, j in pairs:
            w *= np.trace(model.S @ walk(i + 1, j, model.B[rho[i], b[j], b[i]]))
        total += w
    return float(total)


def tensor_brute_logz(prob, model, code: dict) -> float:
    """log of sum over codon assignments c and all structures of
    exp(sum_a theta1[a][c_a]) * tensor_structure_weight."""
    prot = prob.prot
    n = 3 * len(prot)
    sts = all_structures(n)
    Z = 0.0
    for c in itertools.product(*[range(len(code[ch])) for ch in prot]):
        seq = "".join(code[ch][s] for ch, s in zip(prot, c))
        lw = sum(prob.theta1[a][s] for a, s in enumerate(c)) if prob.theta1 is not None else 0.0
        Z += math.exp(lw) * sum(tensor_structure_weight(seq, st, model) for st in sts)
    return math.log(Z)


def tensor_fixed_logz(seq: str, model) -> float:
    """log Z of one fixed sequence by the recursion of SI S2c (eq.
    complicated-pf): Q[i][j+1] = Q[i][j] V_j + sum_k sum_rho Q[i][k]
    B_{k,j} Tr[S B_{j,k} Q[k+1][j]], Q[i][i] = I, Z = Tr[S Q[0][n]]; each
    Q[i][j] carries a scale so that long sequences stay in range."""
    b = [BASES.index(ch) for ch in seq]
    n = len(seq)
    g = model.gamma
    Q = {}
    L = {}  # log scale of Q[i][j]
    for i in range(n + 1):
        Q[i, i] = np.eye(g)
        L[i, i] = 0.0
    for d in range(1, n + 1):
        for i in range(0, n - d + 1):
            j1 = i + d  # Q[i][j1] with j = j1 - 1 the new last base
            j = j1 - 1
            terms = [(Q[i, j] @ model.V[b[j]], L[i, j])]
            for k in range(i, j - 3):
                for r in range(model.xi):
                    t = np.trace(model.S @ model.B[r, b[j], b[k]] @ Q[k + 1, j])
                    if t != 0.0:
                        terms.append((Q[i, k] @ model.B[r, b[k], b[j]] * t, L[i, k] + L[k + 1, j]))
            mx = max(l for _, l in terms)
            M = sum(x * math.exp(l - mx) for x, l in terms)
            s = np.abs(M).max()
            Q[i, j1] = M / s
            L[i, j1] = mx + math.log(s)
    return math.log(np.trace(model.S @ Q[0, n])) + L[0, n]
