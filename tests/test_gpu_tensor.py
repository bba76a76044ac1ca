"""The tensor-based model's sequence-summed free energy (Sections 3b-3c,
Alg. fast-pf) through the C-ABI, against the oracle (oracle/tensor.c).

Every codon boundary of one pass gives a full partition function (the
protein's prefixes), so each case compares m values element by element.
FP64: both sides add positive terms in different orders (the propagation sums
k in 16-wide MFMA groups and 1024-wide chunks), so log Z agrees to a few ulps
per accumulation level: 1e-11 relative is asked.  FP32: every value is a sum
of positive terms, each rounding is at most 2^-24 relative and the pass
nests about n such sums, so |d log Z| <= n * 2^-24 * c; c = 8 covers the
summation depth inside one column (asked: 5e-7 * n absolute, the bound with
n the nucleotide count of the prefix).  300 and 900 nt compare with values
stored by tests/golden/make_oracle_goldens.py (calls only the oracle)."""
import os

import numpy as np
import pytest

import oracle
from paper_2604_19718_amd import binding as B
from paper_2604_19718_amd import inputs as I

from golden.make_oracle_goldens import load_tensor, tensor_path_for

pytestmark = pytest.mark.gpu


def _handle(prec):
    return B.cdz_create(I.energy_tables(1), prec)


def _tol(prec, ref, n):
    return 1e-11 * np.maximum(1.0, np.abs(ref)) if prec == "fp64" else 5e-7 * n


# ("LS", 16, 4): in FP64 the model no longer fits in LDS beside the fold's
# arrays, so the fold reads it from memory (the unstaged variant); ("GAS", 16, 1)
# has 64-wide column blocks (four 16-wide MFMA column tiles)
CASES = [("M", 9, 1), ("MW", 4, 2), ("GCAR", 9, 1), ("MKWLRSGCAT", 9, 1), ("LLLSSSRRR", 9, 2),
         ("ACDEFGHIKLMNPQRSTVWYACDEFGHIKL", 9, 1), ("KWY", 1, 1), ("GAS", 16, 1), ("VVVPC", 3, 4),
         ("LSW", 16, 4)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("prot,gamma,xi", CASES)
def test_tensor_against_oracle_small(prot, gamma, xi, prec):
    prob = I.Problem(prot, I.theta1(5, prot, 0.5), None)
    model = I.tensor_model(7, gamma=gamma, xi=xi, pair=1.5)
    ref, rpre = oracle.tensor_logz(prob, model)
    h = _handle(prec)
    got, gpre = B.cdz_tensor_logz(h, model, prob)
    print(prot, gamma, xi, prec, got, ref, flush=True)
    n = 3 * np.arange(1, len(prot) + 1)
    assert np.all(np.abs(gpre - rpre) <= _tol(prec, rpre, n))
    assert got == gpre[-1]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("m", [40, 100])
def test_tensor_against_oracle_tiles(m, prec):
    """40 residues: two 1024-wide chunks of k, ~28 row tiles; 100 residues
    (300 nt, about 4450 rows): five chunks, a ragged last tile and chunk."""
    prob, model = I.tensor_workload(2, m=m)
    ref, rpre = oracle.tensor_logz(prob, model)
    got, gpre = B.cdz_tensor_logz(_handle(prec), model, prob)
    print(m, prec, got, ref, np.abs(gpre - rpre).max(), flush=True)
    n = 3 * np.arange(1, m + 1)
    assert np.all(np.abs(gpre - rpre) <= _tol(prec, rpre, n))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tensor_against_stored_oracle_900nt(prec):
    if not os.path.exists(tensor_path_for(3)):
        pytest.skip("stored oracle tensor-model values not written")
    prob, model = I.tensor_workload(3)
    ref = load_tensor(3)
    got, gpre = B.cdz_tensor_logz(_handle(prec), model, prob)
    rpre = ref["prefix"]
    err = np.abs(gpre - rpre)
    print(prec, got, float(ref["logz"]), err.max(), flush=True)
    n = 3 * np.arange(1, prob.m + 1)
    assert np.all(err <= _tol(prec, rpre, n))


def test_tensor_errors():
    prob, model = I.tensor_workload(1)
    h = _handle("fp32")
    with pytest.raises(B.CdzError) as e:
        B.cdz_tensor_logz(h, model, I.Problem(prob.prot, prob.theta1, np.zeros((prob.m, 6, 6))))
    assert e.value.status == 1
    with pytest.raises(B.CdzError) as e:
        B.cdz_tensor_logz(h, model, I.Problem("MKZ", None, None))
    assert e.value.status == 2
    bad = I.tensor_model(3)
    bad.S[0, 0] = -1.0
    with pytest.raises(B.CdzError) as e:
        B.cdz_tensor_logz(h, bad, prob)
    assert e.value.status == 3
    big = I.tensor_model(3, gamma=17)
    with pytest.raises(B.CdzError) as e:
        B.cdz_tensor_logz(h, big, prob)
    assert e.value.status == 1
    # the handle still works afterwards
    lz, _ = B.cdz_tensor_logz(h, model, prob)
    assert np.isfinite(lz)


def test_tensor_largest_3900nt():
    """The 1300-residue protein (3900 nt, about 56 700 rows of Q, 28 chunks of
    k in the last columns): FP64 prefix values of its first 100 residues equal
    the oracle's pass over that prefix, FP32 agrees with FP64 at every prefix
    within the FP32 bound, and log Z grows with the prefix."""
    prob, model = I.tensor_workload(5)
    g64, p64 = B.cdz_tensor_logz(_handle("fp64"), model, prob)
    g32, p32 = B.cdz_tensor_logz(_handle("fp32"), model, prob)
    sub = I.Problem(prob.prot[:100], prob.theta1[:100], None)
    ref, rpre = oracle.tensor_logz(sub, model)
    print("3900 nt", g64, g32, np.abs(p32 - p64).max(), np.abs(p64[:100] - rpre).max(), flush=True)
    assert np.all(np.abs(p64[:100] - rpre) <= 1e-11 * np.maximum(1.0, np.abs(rpre)))
    n = 3 * np.arange(1, prob.m + 1)
    assert np.all(np.abs(p32 - p64) <= 5e-7 * n)
    assert np.all(np.diff(p64) > 0)
