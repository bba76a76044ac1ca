"""Frequency matching (Section S4e) through the C-ABI against the oracle.

Small proteins: the oracle runs in the test (FP64 iterates agree to the
rounding of the marginals).  300 and 900 nt: the oracle's runs stored by
tests/golden/make_oracle_goldens.py (calls only the oracle), with the target
bonuses the workloads' codon weights were drawn from, r_tol 0.002 and
unlimited Anderson history, as in the paper's runs.

Tolerances.  FP64 marginals agree with the oracle to ~1e-12; 10-15 least-
squares steps with moderately conditioned differences amplify that by far
less than 1e4, so errors per evaluation and bonuses are compared at 1e-7
relative.  FP32 marginals carry ~1e-6 absolute error; the iterates are then
compared at 1e-3 (relative, bonuses normalised per letter) while the error
sequences agree to 1e-3 absolute and the run meets the same r_tol.
"""
import math
import os

import numpy as np
import pytest

from oracle import freqmatch as FM
from paper_2604_19718_amd import binding as B
from paper_2604_19718_amd import inputs as I

from golden.make_oracle_goldens import FREQ, freq_path_for, load_freq

pytestmark = pytest.mark.gpu


def _norm(f, prot):
    """Bonuses normalised per letter (the ensemble fixes them up to one factor each)."""
    out = np.zeros_like(f)
    for L in set(prot):
        r, d = ord(L) - 65, I.AA_DEGENERACY[L]
        out[r, :d] = f[r, :d] / f[r, :d].sum()
    return out


@pytest.mark.parametrize("m,history", [(6, -1), (12, -1), (12, 2), (20, 0)])
def test_small_fp64_against_oracle(m, history):
    prot = I.protein(40 + m, m)
    en = I.energy_tables(1002)
    if history == 0:  # the plain iteration converges without folding only
        en.hairpin[:] = [math.inf] * 31
    prob = I.Problem(prot, None, I.theta2(6, prot, 0.3))
    ft = I.bonus_targets(77)
    f_o, e_o, ok_o = FM.match_frequencies(prob, en, ft, r_tol=1e-8, max_eval=60, history=history)
    h = B.cdz_create(en, "fp64")
    f_g, e_g, ok_g = B.cdz_match_frequencies(h, prob, ft, r_tol=1e-8, max_eval=60, history=history)
    print(m, history, "evals", len(e_o), len(e_g), flush=True)
    assert ok_o and ok_g and len(e_g) == len(e_o)
    np.testing.assert_allclose(e_g, e_o, rtol=1e-7, atol=1e-12)
    np.testing.assert_allclose(f_g, f_o, rtol=1e-7, atol=0)


def _golden_case(k):
    if not os.path.exists(freq_path_for(k)):
        pytest.skip(f"stored oracle frequency matching for workload {k} not written")
    prob, en = I.workload(k)
    ref = load_freq(k)
    assert int(ref["n"]) == prob.n
    return prob, en, ref


@pytest.mark.parametrize("k", [2, 3])
def test_fp64_against_stored_oracle(k):
    prob, en, ref = _golden_case(k)
    ft = I.bonus_targets(I.config_seed(k))
    h = B.cdz_create(en, "fp64")
    f, errs, ok = B.cdz_match_frequencies(h, prob, ft, r_tol=float(ref["r_tol"]),
                                          max_eval=int(ref["max_eval"]), history=int(ref["history"]))
    print(k, "evals", len(errs), "oracle", len(ref["errs"]), "errs", errs, flush=True)
    assert ok == bool(ref["converged"]) and len(errs) == len(ref["errs"])
    np.testing.assert_allclose(errs, ref["errs"], rtol=1e-7, atol=1e-12)
    np.testing.assert_allclose(f, ref["f"], rtol=1e-7, atol=0)


@pytest.mark.parametrize("k", [2, 3])
def test_fp32_against_stored_oracle(k):
    prob, en, ref = _golden_case(k)
    ft = I.bonus_targets(I.config_seed(k))
    h = B.cdz_create(en, "fp32")
    f, errs, ok = B.cdz_match_frequencies(h, prob, ft, r_tol=float(ref["r_tol"]),
                                          max_eval=int(ref["max_eval"]), history=int(ref["history"]))
    print(k, "evals", len(errs), "oracle", len(ref["errs"]), "errs", errs, flush=True)
    assert ok and errs[-1] < float(ref["r_tol"])
    nc = min(len(errs), len(ref["errs"]))
    np.testing.assert_allclose(errs[:nc], ref["errs"][:nc], rtol=0, atol=1e-3)
    if len(errs) == len(ref["errs"]):
        np.testing.assert_allclose(_norm(f, prob.prot), _norm(ref["f"], prob.prot), rtol=1e-3, atol=0)


def test_rejects_bad_arguments():
    prob, en = I.workload(1)
    h = B.cdz_create(en, "fp64")
    ft = I.bonus_targets(5)
    bad = ft.copy()
    L = prob.prot[0]
    bad[ord(L) - 65, 0] = 0.0
    with pytest.raises(B.CdzError) as e:
        B.cdz_match_frequencies(h, prob, bad)
    assert e.value.status == 1  # CDZ_ERR_ARG
    with pytest.raises(B.CdzError) as e:
        B.cdz_match_frequencies(h, prob, ft, max_eval=0)
    assert e.value.status == 1
    with pytest.raises(B.CdzError) as e:
        B.cdz_match_frequencies(h, I.Problem("MKZ", None, None), ft)
    assert e.value.status == 2  # CDZ_ERR_PROTEIN
    # bonuses of absent letters are never read (NaN there is fine)
    ok = ft.copy()
    absent = [L for L in I.AA_ORDER if L not in prob.prot]
    ok[ord(absent[0]) - 65, :] = np.nan
    f, errs, conv = B.cdz_match_frequencies(h, prob, ok, max_eval=3)
    assert np.all(f[ord(absent[0]) - 65] == 0.0) and len(errs) >= 1


def test_not_converged_reports_last_evaluation():
    prob, en = I.workload(2, m=30)
    ft = I.bonus_targets(I.config_seed(2))
    h = B.cdz_create(en, "fp64")
    f2, e2, ok2 = B.cdz_match_frequencies(h, prob, ft, r_tol=1e-12, max_eval=2)
    assert not ok2 and len(e2) == 2
    f3, e3, _ = B.cdz_match_frequencies(h, prob, ft, r_tol=1e-12, max_eval=3)
    np.testing.assert_allclose(e3[:2], e2, rtol=1e-14)
    # the second evaluation's bonuses are the plain step from the first: f* b*/b
    p = I.Problem(prob.prot, None, prob.theta2)
    f1, e1, _ = B.cdz_match_frequencies(h, p, ft, r_tol=1e-12, max_eval=1)
    mask = FM.present_mask(prob.prot)
    np.testing.assert_allclose(f1[mask], ft[mask], rtol=1e-15)
    assert np.all(f2[~mask] == 0.0)
