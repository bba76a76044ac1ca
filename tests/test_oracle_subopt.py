"""Pins of the suboptimal-state enumeration of the oracle (oracle/mfe.c
``orc_subopt``; SI S4d: every state whose energy lies within a gap of the
minimum).

* Brute force at 1-4 residues (every codon assignment x every structure,
  energies by the Python loop evaluator of oracle/brute.py): the enumerated set
  is exactly the set of states with energy <= MFE + gap, each once, with its
  energy; with an unbounded gap that is every state of the ensemble.
* At 30-60 residues: each returned state has the returned energy under the
  loop evaluator, no state repeats, the smallest energy is the MFE, the argmin
  traceback's state is among them, and the states of a smaller gap are exactly
  those of a larger gap with energy within the smaller one.
* A planted mistake (the depth-first search not restoring its pending stack)
  breaks the unbounded-gap pin.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2604_19718_amd import inputs as I


def _prob(prot, seed=5):
    return I.Problem(prot, I.theta1(seed, prot, 0.5), I.theta2(seed, prot, 0.3))


def _multiloop_energy():
    en = I.energy_tables(1001).copy()
    en.ml_a, en.ml_b = -15.0, -2.0
    en.hairpin[:] = [x - 6.0 for x in en.hairpin]
    return en


def _all_states(prob, en, code):
    out = {}
    for c in itertools.product(*[range(len(code[ch])) for ch in prob.prot]):
        seq = "".join(code[ch][s] for ch, s in zip(prob.prot, c))
        lw = brute.log_weight(prob, c)
        for st in brute.structures(seq):
            pt = [-1] * len(seq)
            for i, j in st:
                pt[i], pt[j] = j, i
            out[(tuple(c), tuple(pt))] = brute.loop_energy(seq, st, en) - lw
    return out


def _keys(C, P):
    return [(tuple(int(x) for x in c), tuple(int(x) for x in p)) for c, p in zip(C, P)]


def _check_against_brute(prob, en, gap, code):
    allst = _all_states(prob, en, code)
    mn = min(allst.values())
    want = {k for k, e in allst.items() if e <= mn + gap + 1e-9 * max(1.0, abs(mn))}
    mfe, E, C, P, complete = oracle.subopt(prob, en, gap, max_states=50000)
    keys = _keys(C, P)
    assert complete and abs(mfe - mn) <= 1e-12 * max(1.0, abs(mn))
    assert len(keys) == len(set(keys)) == len(want) and set(keys) == want
    for k, e in zip(keys, E):
        assert abs(allst[k] - e) <= 1e-12 * max(1.0, abs(e))
    return len(allst), len(want)


CASES = [("M", "default", 2.0), ("KW", "default", 3.0), ("GCAR", "default", 1.5), ("CYHW", "interior", 5.0),
         ("MKWL", "bulge", 6.0), ("GCGR", "multiloop", 3.0), ("CYHW", "default", 0.0)]


def _energy(kind):
    return {"default": I.energy_tables(1001), "multiloop": _multiloop_energy(),
            "interior": I.interior_rich_energy(7), "bulge": I.bulge_rich_energy(7)}[kind]


@pytest.mark.parametrize("prot,kind,gap", CASES)
def test_subopt_brute_force(prot, kind, gap, genetic_code):
    _check_against_brute(_prob(prot), _energy(kind), gap, genetic_code)


@pytest.mark.parametrize("prot,kind", [("GCAR", "default"), ("VVVP", "multiloop"), ("RSL", "default")])
def test_subopt_every_state(prot, kind, genetic_code):
    """An unbounded gap enumerates the whole ensemble, each state once."""
    total, got = _check_against_brute(_prob(prot), _energy(kind), 1e6, genetic_code)
    assert got == total


@pytest.mark.parametrize("m,gap", [(30, 1.0), (60, 0.5)])
def test_subopt_larger(m, gap, genetic_code):
    prob, en = I.workload(2, m=m)
    mfe, E, C, P, complete = oracle.subopt(prob, en, gap, max_states=20000)
    assert complete and len(E) >= 1
    keys = _keys(C, P)
    assert len(set(keys)) == len(keys)
    assert abs(E.min() - mfe) <= 1e-9 * abs(mfe) and np.all(E <= mfe + gap + 1e-9 * abs(mfe))
    for (c, p), e in zip(keys[:200], E[:200]):
        seq = "".join(genetic_code[ch][s] for ch, s in zip(prob.prot, c))
        pl = [(i, j) for i, j in enumerate(p) if j > i]
        assert abs(brute.loop_energy(seq, pl, en) - brute.log_weight(prob, list(c)) - e) <= 1e-9 * abs(e)
    v, cod, pairs = oracle.mfe(prob, en)
    assert (tuple(int(x) for x in cod), tuple(int(x) for x in pairs)) in set(keys)
    # nested gaps
    mfe2, E2, C2, P2, _ = oracle.subopt(prob, en, gap / 2, max_states=20000)
    sub = {k for k, e in zip(keys, E) if e <= mfe + gap / 2 + 1e-9 * abs(mfe)}
    assert set(_keys(C2, P2)) == sub


def test_subopt_limit_and_errors():
    prob, en = I.workload(2, m=30)
    _, E, C, P, complete = oracle.subopt(prob, en, 1.0, max_states=3)
    assert not complete and len(E) == 3
    _, E2, _, _, _ = oracle.subopt(prob, en, 1.0, max_states=20000)
    assert np.array_equal(E, E2[:3])  # the first states of the same depth-first order
    for gap in (-1.0, float("nan")):
        with pytest.raises(RuntimeError):
            oracle.subopt(prob, en, gap)


def test_planted_no_restore_is_caught(tmp_path, genetic_code):
    path = oracle.build_variant(str(tmp_path / "lib_norestore.so"), ["PLANT_SUBOPT_NO_RESTORE"])
    bad = oracle.load(path)
    caught = False
    try:
        oracle.use(bad)
        try:
            _check_against_brute(_prob("GCAR"), _energy("default"), 1e6, genetic_code)
        except (AssertionError, RuntimeError):
            caught = True
    finally:
        oracle.use(None)
    assert caught
