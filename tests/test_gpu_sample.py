"""GPU traceback sampler against the oracle sampler and exact distributions."""
import collections
import math
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2604_19718_amd import binding as B
from paper_2604_19718_amd import inputs as I

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("prot", ["M", "KLV", "MKWLRS", "GASCYHWQ"])
def test_fp64_samples_match_oracle_draw_for_draw(prot):
    """Same seed, same protocol: identical codons and structures (FP64)."""
    en = I.energy_tables(1001)
    prob = I.Problem(prot, I.theta1(5, prot), I.theta2(5, prot))
    seed = 0x1234567890ABCDEF
    oc, op = oracle.sample(prob, en, seed, 200)
    h = B.cdz_create(en, "fp64")
    gc, gp = B.cdz_sample(h, prob, seed, 200)
    mism = int(np.sum(np.any(oc != gc, axis=1) | np.any(op != gp, axis=1)))
    print(prot, "mismatching samples", mism, flush=True)
    assert mism == 0


def test_fp64_samples_workload_8aa_and_100aa():
    for k, m, N in ((1, None, 100), (2, 60, 100)):
        prob, en = I.workload(k, m=m)
        seed = I.sampler_seed(k)
        oc, op = oracle.sample(prob, en, seed, N)
        gc, gp = B.cdz_sample(B.cdz_create(en, "fp64"), prob, seed, N)
        mism = int(np.sum(np.any(oc != gc, axis=1) | np.any(op != gp, axis=1)))
        print("workload", k, m, "mismatching samples", mism, flush=True)
        assert mism == 0


@pytest.mark.parametrize("model", ["bulge_rich", "interior_rich"])
def test_fp64_samples_loop_rich_models(model):
    """Draw for draw under tables where long bulges and interior loops are
    frequent, so that every window branch of the pair decision is taken."""
    en = getattr(I, f"{model}_energy")(7)
    prob, _ = I.workload(2, m=40)
    seed = I.sampler_seed(2, 1)
    oc, op = oracle.sample(prob, en, seed, 200)
    gc, gp = B.cdz_sample(B.cdz_create(en, "fp64"), prob, seed, 200)
    mism = int(np.sum(np.any(oc != gc, axis=1) | np.any(op != gp, axis=1)))
    print(model, "mismatching samples", mism, flush=True)
    assert mism == 0


def _joint_tv(cod, pairs, joint):
    N = len(cod)
    cnt = collections.Counter()
    for k in range(N):
        pt = pairs[k]
        st = tuple((i, int(pt[i])) for i in range(len(pt)) if pt[i] > i)
        cnt[(tuple(int(x) for x in cod[k]), st)] += 1
    known = {(c, st) for c, st, _ in joint}
    assert all(key in known for key in cnt)
    return 0.5 * sum(abs(cnt.get((c, st), 0) / N - pr) for c, st, pr in joint)


@pytest.mark.parametrize("prot", ["KLV", "RSLW"])
def test_fp32_joint_distribution(prot):
    code = brute.load_genetic_code(os.path.join(GOLDEN, "genetic_code.txt"))
    en = I.energy_tables(1001)
    prob = I.Problem(prot, I.theta1(13, prot), I.theta2(13, prot))
    ref = brute.enumerate_ensemble(prob, en, code)
    N = 200_000
    cod, pairs = B.cdz_sample(B.cdz_create(en, "fp32"), prob, 777, N)
    tv = _joint_tv(cod, pairs, ref["joint"])
    bound = 3 * math.sqrt(len(ref["joint"]) / (2 * math.pi * N))
    print(prot, "TV", tv, "bound", bound, flush=True)
    assert tv <= bound


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_marginal_frequencies_300nt(prec):
    prob, en = I.workload(2)
    h = B.cdz_create(en, prec)
    ref = B.cdz_marginals(h, prob)
    N = 2000
    cod, pairs = B.cdz_sample(h, prob, 31337, N)
    freq = np.zeros((prob.m, 6))
    for a in range(prob.m):
        freq[a] = np.bincount(cod[:, a], minlength=6)[:6] / N
    p = np.clip(ref["codon"], 0, 1)
    z = np.abs(freq - p) - 5 * np.sqrt(p * (1 - p) / N) - 3.0 / N  # rare codons are discrete
    assert z.max() <= 0, z.max()
    n = prob.n
    pf = np.zeros((n, n))
    for k in range(N):
        pt = pairs[k]
        idx = np.where(pt >= 0, pt, np.arange(n))
        pf[np.arange(n), idx] += 1.0 / N
    P = np.clip(ref["pair"], 0, 1)
    z = np.abs(pf - P) - 5 * np.sqrt(P * (1 - P) / N) - 2.0 / N
    assert z.max() <= 0, z.max()
