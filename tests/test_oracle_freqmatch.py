"""Pins of the frequency-matching oracle (Section S4e, algorithm "iterative",
with Anderson acceleration after Walker and Ni 2011).

* Anderson on a linear contraction g(x) = Mx + c: with the whole history it is
  a Krylov method (equivalent to GMRES on (I - M)x = c), so it reaches the
  exact fixed point (I - M)^-1 c within dim + 1 evaluations; the plain
  iteration (history 0) contracts by at most ||M|| per evaluation.
* No folding (every hairpin forbidden, so no structure has a pair) and no
  codon-pair weights: the codon marginals are f / sum f per residue, so the
  target bonuses already match (error 0 at the first evaluation).
* No folding with codon-pair weights: the ensemble is a chain of codons whose
  marginals follow from the forward-backward recursion written out here; the
  matched bonuses must reproduce b* under that independent computation.
* Brute force at 3-4 residues with folding: matching through the oracle's
  marginals and through enumeration of every (codon sequence, structure)
  gives the same iterates, and the final bonuses meet the tolerance under
  enumeration.
* Planted mistakes (update sign of the printed algorithm, slot transposed in
  the accumulation, target not normalised per residue) fail these pins.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from oracle import freqmatch as FM
from paper_2604_19718_amd import inputs as I


def _no_fold(seed=7):
    en = I.energy_tables(seed)
    en.hairpin[:] = [math.inf] * 31
    return en


def _f_target(prot, seed=3):
    """Bonuses exp(theta1 type weights): the weights a soft constraint was built from."""
    t1 = I.theta1(seed, prot, 0.5)
    f = np.zeros((FM.NLET, FM.NSLOT))
    for a, L in enumerate(prot):
        d = FM.degeneracy(L)
        f[ord(L) - 65, :d] = np.exp(t1[a, :d])
    return f


def test_degeneracy_is_the_genetic_code():
    assert sum(FM.degeneracy(L) for L in I.AA_ORDER) == 61
    for L in I.AA_ORDER:
        assert FM.degeneracy(L) == I.AA_DEGENERACY[L]


@pytest.mark.parametrize("dim", [3, 6, 9])
def test_anderson_linear_terminates(dim):
    rng = np.random.default_rng(dim)
    M = rng.standard_normal((dim, dim))
    M *= 0.9 / np.linalg.norm(M, 2)
    c = rng.standard_normal(dim)
    xstar = np.linalg.solve(np.eye(dim) - M, c)
    x, errs, ok = FM.anderson(lambda v: M @ v + c, np.zeros(dim), 1e-10, dim + 2, history=-1)
    assert ok and len(errs) <= dim + 2
    np.testing.assert_allclose(x, xstar, atol=1e-9)
    # plain iteration: residual contracts by at most ||M||_2 (<= sqrt(dim) in the max norm)
    x0, errs0, _ = FM.anderson(lambda v: M @ v + c, np.zeros(dim), 0.0, 12, history=0)
    r0 = np.linalg.norm(c)
    for k, e in enumerate(errs0):
        assert e <= 0.9 ** k * r0 * math.sqrt(dim) * (1 + 1e-12) + 1e-15
    assert errs0[-1] > errs[-1]


def test_no_folding_target_is_fixed_point():
    prot = I.protein(11, 25)
    prob = I.Problem(prot, None, None)
    f0 = _f_target(prot)
    f, errs, ok = FM.match_frequencies(prob, _no_fold(), f0, r_tol=1e-10, max_eval=3)
    assert ok and len(errs) == 1 and errs[0] < 1e-12
    mask = FM.present_mask(prot)
    np.testing.assert_allclose(f[mask], f0[mask], rtol=1e-14)


def _chain_codon_marginals(prot, x, theta2):
    """Codon marginals of a chain of codons (no folding): node weights exp(x),
    edge weights exp(theta2[a][s][t]); forward-backward recursion."""
    m = len(prot)
    deg = [FM.degeneracy(L) for L in prot]
    node = [np.exp(x[ord(L) - 65, :deg[a]]) for a, L in enumerate(prot)]
    edge = [None] + [np.exp(theta2[a][:deg[a - 1], :deg[a]]) for a in range(1, m)]
    fw = [node[0] / node[0].sum()]
    for a in range(1, m):
        v = (fw[-1] @ edge[a]) * node[a]
        fw.append(v / v.sum())
    bw = [None] * m
    bw[m - 1] = np.ones(deg[m - 1])
    for a in range(m - 2, -1, -1):
        v = edge[a + 1] @ (node[a + 1] * bw[a + 1])
        bw[a] = v / v.sum()
    out = np.zeros((m, 6))
    for a in range(m):
        p = fw[a] * bw[a]
        out[a, :deg[a]] = p / p.sum()
    return out


def test_no_folding_with_pair_weights_matches_chain():
    prot = I.protein(12, 30)
    t2 = I.theta2(5, prot, 0.6)
    prob = I.Problem(prot, None, t2)
    en = _no_fold()
    f0 = _f_target(prot)
    # the oracle's marginals equal the chain's in this case
    x0 = np.zeros((FM.NLET, FM.NSLOT))
    x0[f0 > 0] = np.log(f0[f0 > 0])
    got = oracle.marginals(I.Problem(prot, FM.theta1_of(prot, x0), t2), en)["codon"]
    np.testing.assert_allclose(got, _chain_codon_marginals(prot, x0, t2), atol=1e-13)
    f, errs, ok = FM.match_frequencies(prob, en, f0, r_tol=1e-9, max_eval=40)
    assert ok and errs[0] > 1e-2
    x = np.zeros((FM.NLET, FM.NSLOT))
    x[f > 0] = np.log(f[f > 0])
    b = FM.achieved_frequencies(prot, _chain_codon_marginals(prot, x, t2))
    bs = FM.target_frequencies(prot, f0)
    mask = FM.present_mask(prot)
    assert np.max(np.abs(np.log(b[mask] / bs[mask]))) < 1e-9


def _brute_marg(code):
    return lambda p, e: brute.enumerate_ensemble(p, e, code)["codon"]


@pytest.mark.parametrize("prot", ["KLV", "GASR", "CYHW"])
def test_brute_force_matching(prot, genetic_code):
    en = I.energy_tables(1001)
    t2 = I.theta2(5, prot, 0.3)
    prob = I.Problem(prot, None, t2)
    f0 = _f_target(prot, seed=9)
    f_o, e_o, ok_o = FM.match_frequencies(prob, en, f0, r_tol=1e-9, max_eval=40)
    f_b, e_b, ok_b = FM.match_frequencies(prob, en, f0, r_tol=1e-9, max_eval=40,
                                          marg=_brute_marg(genetic_code))
    assert ok_o and ok_b and len(e_o) == len(e_b)
    np.testing.assert_allclose(e_o, e_b, rtol=1e-8, atol=1e-12)
    np.testing.assert_allclose(f_o, f_b, rtol=1e-9)
    x = np.zeros((FM.NLET, FM.NSLOT))
    x[f_o > 0] = np.log(f_o[f_o > 0])
    ref = brute.enumerate_ensemble(I.Problem(prot, FM.theta1_of(prot, x), t2), en, genetic_code)["codon"]
    b = FM.achieved_frequencies(prot, ref)
    bs = FM.target_frequencies(prot, f0)
    mask = FM.present_mask(prot)
    assert np.max(np.abs(np.log(b[mask] / bs[mask]))) < 1e-9


def test_anderson_and_plain_reach_the_same_frequencies():
    """Without folding the plain iteration converges too (with folding at these
    energies it can cycle, which is why the acceleration is used); both reach the
    same frequencies, Anderson in fewer evaluations."""
    prot = I.protein(12, 30)
    prob = I.Problem(prot, None, I.theta2(6, prot, 0.6))
    en = _no_fold()
    f0 = _f_target(prot)
    fa, ea, oka = FM.match_frequencies(prob, en, f0, r_tol=1e-9, max_eval=60, history=-1)
    fp, ep, okp = FM.match_frequencies(prob, en, f0, r_tol=1e-9, max_eval=200, history=0)
    assert oka and okp
    assert len(ea) < len(ep)
    # bonuses are fixed up to one factor per residue letter: compare per-letter normalised
    for L in set(prot):
        r, d = ord(L) - 65, FM.degeneracy(L)
        np.testing.assert_allclose(fa[r, :d] / fa[r, :d].sum(), fp[r, :d] / fp[r, :d].sum(), rtol=1e-7)


# ---- planted mistakes: each must break a pin above

def _chain_case():
    prot = I.protein(12, 30)
    return prot, I.theta2(5, prot, 0.6), _no_fold(), _f_target(prot)


def _chain_pin_holds(prot, t2, en, f0, f, ok):
    """Frequencies of the chain under bonuses f against b*, both formed here
    (not through the oracle's helpers, which a plant may have replaced)."""
    if not ok:
        return False
    x = np.zeros((FM.NLET, FM.NSLOT))
    x[f > 0] = np.log(f[f > 0])
    cm = _chain_codon_marginals(prot, x, t2)
    worst = 0.0
    for L in set(prot):
        r, d = ord(L) - 65, I.AA_DEGENERACY[L]
        idx = [a for a, c in enumerate(prot) if c == L]
        b = cm[idx, :d].sum(axis=0)
        bs = len(idx) * f0[r, :d] / f0[r, :d].sum()
        worst = max(worst, float(np.max(np.abs(np.log(b / bs)))))
    return worst < 1e-9


def _planted_breaks_pin(**kw):
    """Run the chain case with a planted mistake in place; True when the pin fails
    (no convergence, a run-away rejected by the oracle, or wrong frequencies)."""
    prot, t2, en, f0 = _chain_case()
    try:
        with np.errstate(all="ignore"):
            f, errs, ok = FM.match_frequencies(I.Problem(prot, None, t2), en, f0, r_tol=1e-9, max_eval=40, **kw)
    except RuntimeError:
        return True
    return not _chain_pin_holds(prot, t2, en, f0, f, ok)


def test_planted_printed_update_sign(monkeypatch):
    real = FM.anderson

    def flipped(g, x0, tol, max_eval, history=-1, norm=None):
        return real(lambda x: 2 * x - g(x), x0, tol, max_eval, history)  # x - r instead of x + r
    monkeypatch.setattr(FM, "anderson", flipped)
    # the plain iteration runs away from the target; with the whole history the
    # least-squares step finds the same root of r either way, so only history 0
    # tells the two readings apart
    assert _planted_breaks_pin(history=0)


def test_planted_slot_transpose(monkeypatch):
    real = FM.achieved_frequencies
    monkeypatch.setattr(FM, "achieved_frequencies", lambda p, c: real(p, c[:, ::-1]))
    assert _planted_breaks_pin()


def test_planted_unnormalised_target(monkeypatch):
    def raw(p, f):
        b = np.zeros((FM.NLET, FM.NSLOT))
        for L in set(p):
            r, d = ord(L) - 65, FM.degeneracy(L)
            b[r, :d] = p.count(L) * f[r, :d]
        return b
    monkeypatch.setattr(FM, "target_frequencies", raw)
    assert _planted_breaks_pin()
