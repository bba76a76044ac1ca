"""Pins of the minimum-free-energy oracle (oracle/mfe.c; Section 4d, the
(min, +) evaluation algebra of SI S2c).

* Brute force (every codon assignment x every structure, energies by the
  Python loop evaluator of oracle/brute.py) at 1-4 residues: the minimum and
  the minimising state.
* Per-sequence brute force at 5-6 residues of low degeneracy: the minimum
  over codon sequences of (-log W + the minimum over that sequence's
  structures).
* A 12-nt multiloop of two minimal hairpins (tables that favour multiloops)
  against brute force: the tightest split of the recursion.
* The traceback's state at 40-100 residues has exactly the returned energy
  under the Python loop evaluator of oracle/brute.py (written separately from
  both DP implementations), and the MFE bounds log Z of the (+, x) oracle:
  -MFE <= log Z.
* Planted mistakes in mfe.c (split range, codon-pair sign, stack table
  transposed) each break a pin.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2604_19718_amd import inputs as I


def _prob(prot, seed=5, pair=True):
    return I.Problem(prot, I.theta1(seed, prot, 0.5), I.theta2(seed, prot, 0.3) if pair else None)


def _state_energy(prob, en, code, cod, pairs):
    seq = "".join(code[ch][s] for ch, s in zip(prob.prot, cod))
    pl = [(i, j) for i, j in enumerate(pairs) if j > i]
    return brute.loop_energy(seq, pl, en) - brute.log_weight(prob, list(cod))


def _brute_min(prob, en, code):
    best, arg = math.inf, None
    for c in itertools.product(*[range(len(code[ch])) for ch in prob.prot]):
        seq = "".join(code[ch][s] for ch, s in zip(prob.prot, c))
        lw = brute.log_weight(prob, c)
        for st in brute.structures(seq):
            e = brute.loop_energy(seq, st, en) - lw
            if e < best:
                best, arg = e, (c, st)
    return best, arg


@pytest.mark.parametrize("prot", ["M", "KW", "KLV", "GAS", "RSL", "MKWL", "CYHW", "GCAR"])
def test_mfe_brute_force_small(prot, genetic_code):
    en = I.energy_tables(1001)
    prob = _prob(prot)
    ref, (c, st) = _brute_min(prob, en, genetic_code)
    got, cod, pairs = oracle.mfe(prob, en)
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (got, ref)
    # the traceback's state is the brute-force minimiser (no ties at these energies)
    n = 3 * len(prot)
    pt = [-1] * n
    for i, j in st:
        pt[i], pt[j] = j, i
    assert list(cod) == list(c)
    assert list(pairs) == pt


@pytest.mark.parametrize("prot", ["MWKYFC", "DEKMHW", "NQCYFW"])
def test_mfe_per_sequence_brute_force(prot, genetic_code):
    """6 residues (18 nt), low degeneracy: min over codon sequences of
    (-log W + min over structures), structures enumerated per sequence."""
    en = I.interior_rich_energy(3) if prot == "NQCYFW" else I.energy_tables(1002)
    prob = _prob(prot, seed=8)
    best = math.inf
    for c in itertools.product(*[range(len(genetic_code[ch])) for ch in prot]):
        seq = "".join(genetic_code[ch][s] for ch, s in zip(prot, c))
        e = min(brute.loop_energy(seq, st, en) for st in brute.structures(seq))
        best = min(best, e - brute.log_weight(prob, c))
    got, cod, pairs = oracle.mfe(prob, en)
    assert abs(got - best) <= 1e-12 * max(1.0, abs(best))
    assert abs(_state_energy(prob, en, genetic_code, cod, pairs) - got) <= 1e-10


@pytest.mark.parametrize("m,pair", [(40, True), (100, True), (100, False)])
def test_mfe_traceback_energy_and_bound(m, pair, genetic_code):
    prob0, en = I.workload(2, m=m)
    prob = prob0 if pair else I.Problem(prob0.prot, prob0.theta1, None)
    got, cod, pairs = oracle.mfe(prob, en)
    e = _state_energy(prob, en, genetic_code, cod, pairs)
    assert abs(e - got) <= 1e-9 * max(1.0, abs(got)), (e, got)
    assert np.all((pairs == -1) | (pairs[np.maximum(pairs, 0)] == np.arange(len(pairs))))
    lz = oracle.logz(prob, en)
    assert -got <= lz + 1e-9 * abs(lz)
    # and the minimiser carries a real share of the ensemble at these energies
    assert lz + got < 0.5 * abs(lz)


def multiloop_energy():
    """Tables under which short multiloops win: closing and branch terms
    favourable, hairpins 6 kT cheaper."""
    en = I.energy_tables(1001).copy()
    en.ml_a, en.ml_b = -15.0, -2.0
    en.hairpin[:] = [x - 6.0 for x in en.hairpin]
    return en


def test_mfe_brute_force_multiloop(genetic_code):
    """At 12 nt the minimiser is a multiloop of two minimal hairpins, the
    tightest split the recursion allows (u = i + 5)."""
    prob = _prob("VVVP", seed=4)
    en = multiloop_energy()
    ref, (c, st) = _brute_min(prob, en, genetic_code)
    assert sorted(st) == [(0, 11), (1, 5), (6, 10)]
    got, cod, pairs = oracle.mfe(prob, en)
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref))
    assert list(pairs) == [11, 5, -1, -1, -1, 1, 10, -1, -1, -1, 6, 0]


PLANTS = ["PLANT_MFE_SPLIT_RANGE", "PLANT_MFE_PAIR_SIGN", "PLANT_MFE_STACK_SWAP"]


@pytest.mark.parametrize("plant", PLANTS)
def test_planted_mistakes_are_caught(plant, tmp_path, genetic_code):
    path = oracle.build_variant(str(tmp_path / f"lib_{plant}.so"), [plant])
    bad = oracle.load(path)
    caught = False
    try:
        oracle.use(bad)
        cases = [("VVVP", multiloop_energy()), ("CYHW", I.energy_tables(1001)),
                 ("GCAR", I.energy_tables(1003))]
        for prot, en in cases:
            prob = _prob(prot, seed=4)
            got, cod, pairs = oracle.mfe(prob, en)
            oracle.use(None)
            ref, _ = _brute_min(prob, en, genetic_code)
            if abs(got - ref) > 1e-9 * max(1.0, abs(ref)):
                caught = True
            oracle.use(bad)
    finally:
        oracle.use(None)
    assert caught, plant
