"""The oracle's pins catch planted mistakes (CPU only).

Each variant of the oracle is built with one deliberate, plausible mistake
(a swapped table index, a dropped energy term, a transposed weight, an
off-by-one split range, a forgotten adjoint term, a biased sampling
decision) and must fail at least one of the checks the pins rely on:
brute-force enumeration, the sum of single-sequence partition functions,
the adjoint invariants, and the sampler's joint distribution."""
import collections
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2604_19718_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PLANTS = ["PLANT_INNER_MISMATCH", "PLANT_ML_CLOSING", "PLANT_PAIR_TRANSPOSE",
          "PLANT_HAIRPIN_EXTRAP", "PLANT_STACK_SWAP", "PLANT_SPLIT_RANGE",
          "PLANT_REVERSE_EDGE", "PLANT_SAMPLER_BULGE"]


def _lse(v):
    mx = max(v)
    return mx + math.log(sum(math.exp(x - mx) for x in v))


def _checks(code):
    """Yield (name, ok) for each pin; the default oracle passes all of them."""
    en = I.energy_tables(1001)
    for prot in ("KLV", "RSLW", "MKWL"):
        prob = I.Problem(prot, I.theta1(5, prot), I.theta2(5, prot))
        ref = brute.enumerate_ensemble(prob, en, code)
        got = oracle.marginals(prob, en, checks=True)
        ok = abs(got["logz"] - ref["logz"]) < 1e-10
        for k in ("pair", "codon", "codon_pair", "base"):
            ok = ok and np.abs(got[k] - ref[k]).max() < 1e-10
        yield f"brute {prot}", ok
    for prot in ("MWMWKMWMWMWIMWMWMWMWMWMWMWMWMWMWKMWMWC", "KLVSAG"):
        prob = I.Problem(prot, I.theta1(9, prot), I.theta2(9, prot))
        vals = []
        for c in itertools.product(*[range(len(code[ch])) for ch in prot]):
            seq = ["ACGU".index(x) for x in "".join(code[ch][s] for ch, s in zip(prot, c))]
            vals.append(brute.log_weight(prob, c) + oracle.seq_logz(seq, en))
        yield f"sum-of-sequences {len(prot)}", abs(oracle.logz(prob, en) - _lse(vals)) < 1e-9
    prot = "MWMWKMWMWMWIMWMWMWMWMWMWMWMWMWMWKMWMWC"
    prob = I.Problem(prot, I.theta1(9, prot), I.theta2(9, prot))
    eh = I.hairpin_only_energy(1001)
    vals = []
    for c in itertools.product(*[range(len(code[ch])) for ch in prot]):
        seq = ["ACGU".index(x) for x in "".join(code[ch][s] for ch, s in zip(prot, c))]
        vals.append(brute.log_weight(prob, c) + oracle.seq_logz(seq, eh))
    yield "hairpin-only model", abs(oracle.logz(prob, eh) - _lse(vals)) < 1e-10
    prob, _ = I.workload(2, m=30)
    got = oracle.marginals(prob, en, checks=True)
    yield "adjoint invariants", (np.abs(got["vcheck"] - 1).max() < 1e-10 and
                                 np.abs(got["echeck"] - 1).max() < 1e-10)
    # sampler: joint distribution under the interior-loop-rich model
    prot = "RSLWA"
    prob = I.Problem(prot, I.theta1(13, prot), I.theta2(13, prot))
    en = I.interior_rich_energy(1001)
    ref = brute.enumerate_ensemble(prob, en, code)
    N = 100_000
    cod, pairs = oracle.sample(prob, en, 4242, N)
    cnt = collections.Counter()
    for k in range(N):
        pt = pairs[k]
        st = tuple((i, int(pt[i])) for i in range(len(pt)) if pt[i] > i)
        cnt[(tuple(int(x) for x in cod[k]), st)] += 1
    chi2 = sum((cnt.get((c, st), 0) - N * pr) ** 2 / (N * pr) for c, st, pr in ref["joint"] if N * pr > 5)
    dof = sum(1 for _, _, pr in ref["joint"] if N * pr > 5) - 1
    from scipy.stats import chi2 as chi2dist
    yield "sampler chi-square", chi2dist.sf(chi2, dof) > 1e-4


@pytest.fixture(scope="module")
def code():
    return brute.load_genetic_code(os.path.join(GOLDEN, "genetic_code.txt"))


def test_default_oracle_passes_every_check(code):
    oracle.use(None)
    failed = [name for name, ok in _checks(code) if not ok]
    assert not failed, failed


@pytest.mark.parametrize("plant", PLANTS)
def test_planted_mistake_is_caught(plant, code, tmp_path):
    path = oracle.build_variant(str(tmp_path / f"lib_{plant}.so"), [plant])
    oracle.use(oracle.load(path))
    try:
        results = list(_checks(code))
    finally:
        oracle.use(None)
    failed = [name for name, ok in results if not ok]
    print(plant, "caught by", failed)
    assert failed, f"{plant} was not detected by any pin"
