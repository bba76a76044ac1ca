"""Pins of the tensor-model oracle (oracle/tensor.c; Sections 3b-3c, SI S2b-S2c
and Alg. complex-pf with the folding function of eq. design-fold).

* Brute force at 1-4 residues: every codon assignment x every structure (any
  two bases at least 4 apart may pair; the model's B decides the weight), each
  weighed by the loop-product definition of eq. general-model with one rank
  index per pair (oracle/brute.py), xi = 1 and 2, gamma = 4 and 9.
* Fixed sequences (proteins of single-codon residues M and W) up to 60 nt
  against the SI's other recursion, eq. complicated-pf, evaluated in numpy.
* Sum over sequences at 6 low-degeneracy residues: sum over codon sequences
  of the codon bonus times the eq. complicated-pf value.
* No pairs (B = 0) at 100 residues: the transfer-matrix closed form
  Tr[S prod_a sum_c w(c) V_{c1} V_{c2} V_{c3}], built from the genetic code
  and not from the tensor train.
* The prefix values equal log Z of the protein's prefixes.
* Planted mistakes (inner pair side transposed, hairpins of two bases allowed,
  the fold's scale factor dropped) each break a pin.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2604_19718_amd import inputs as I


def _prob(prot, seed=5, bonus=True):
    return I.Problem(prot, I.theta1(seed, prot, 0.5) if bonus else None, None)


@pytest.mark.parametrize("prot,gamma,xi,pair", [
    ("M", 4, 1, 3.0), ("KW", 4, 1, 3.0), ("GCA", 4, 1, 3.0), ("MWK", 4, 2, 3.0), ("CYH", 9, 1, 2.0),
    ("MWCY", 3, 1, 4.0), ("GAS", 3, 2, 4.0)])
def test_tensor_brute_force(prot, gamma, xi, pair, genetic_code):
    prob = _prob(prot)
    model = I.tensor_model(7, gamma=gamma, xi=xi, pair=pair)
    ref = brute.tensor_brute_logz(prob, model, genetic_code)
    got, pre = oracle.tensor_logz(prob, model)
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (got, ref)
    assert pre[-1] == got


@pytest.mark.parametrize("prot,xi", [("MWWMWMMW", 1), ("MWMWWWMMWMWWMMWMWMWW", 1), ("WMMWMWMW", 2)])
def test_tensor_fixed_sequence(prot, xi, genetic_code):
    seq = "".join(genetic_code[c][0] for c in prot)
    model = I.tensor_model(11, gamma=9, xi=xi, pair=1.5)
    ref = brute.tensor_fixed_logz(seq, model)
    got, _ = oracle.tensor_logz(_prob(prot, bonus=False), model)
    assert abs(got - ref) <= 1e-11 * abs(ref), (got, ref)


def test_tensor_sum_over_sequences(genetic_code):
    prot = "MWKCYF"
    prob = _prob(prot, seed=9)
    model = I.tensor_model(12, gamma=9, pair=1.0)
    terms = []
    for c in itertools.product(*[range(len(genetic_code[ch])) for ch in prot]):
        seq = "".join(genetic_code[ch][s] for ch, s in zip(prot, c))
        terms.append(sum(prob.theta1[a][s] for a, s in enumerate(c)) + brute.tensor_fixed_logz(seq, model))
    mx = max(terms)
    ref = mx + math.log(sum(math.exp(t - mx) for t in terms))
    got, _ = oracle.tensor_logz(prob, model)
    assert abs(got - ref) <= 1e-11 * abs(ref)


def test_tensor_no_pairs_closed_form(genetic_code):
    prob, model = I.tensor_workload(2)
    model.B[:] = 0.0
    g = model.gamma
    M = np.eye(g)
    logscale = 0.0
    B = "ACGU"
    for a, ch in enumerate(prob.prot):
        T = np.zeros((g, g))
        for s, cod in enumerate(genetic_code[ch]):
            T += math.exp(prob.theta1[a][s]) * (model.V[B.index(cod[0])] @ model.V[B.index(cod[1])]
                                                 @ model.V[B.index(cod[2])])
        M = M @ T
        sc = np.abs(M).max()
        M /= sc
        logscale += math.log(sc)
    ref = math.log(np.trace(model.S @ M)) + logscale
    got, _ = oracle.tensor_logz(prob, model)
    assert abs(got - ref) <= 1e-11 * abs(ref)


def test_tensor_prefix_values():
    prob, model = I.tensor_workload(2, m=24)
    _, pre = oracle.tensor_logz(prob, model)
    for a in (0, 5, 11, 23):
        sub = I.Problem(prob.prot[:a + 1], prob.theta1[:a + 1], None)
        ref, _ = oracle.tensor_logz(sub, model)
        assert abs(pre[a] - ref) <= 1e-12 * abs(ref)


PLANTS = ["PLANT_TENSOR_INNER_ORDER", "PLANT_TENSOR_HAIRPIN", "PLANT_TENSOR_SCALE"]


@pytest.mark.parametrize("plant", PLANTS)
def test_tensor_planted_mistakes_are_caught(plant, tmp_path, genetic_code):
    path = oracle.build_variant(str(tmp_path / f"lib_{plant}.so"), [plant])
    bad = oracle.load(path)
    caught = []
    try:
        oracle.use(bad)
        for check in (lambda: test_tensor_brute_force("GCA", 4, 1, 3.0, genetic_code),
                      lambda: test_tensor_fixed_sequence("MWMWWWMMWMWWMMWMWMWW", 1, genetic_code)):
            try:
                check()
                caught.append(False)
            except (AssertionError, RuntimeError):
                caught.append(True)
    finally:
        oracle.use(None)
    assert any(caught), plant
