"""The 256-protein batch (lengths uniform in 30..400 residues, per-protein
codon and codon-pair weights, FP32 scaled) in one call, forward + outside +
64 samples each: members equal their single-problem calls bit for bit, the
shortest member matches the oracle, and invariants hold for every member."""
import numpy as np
import pytest

import oracle
from paper_2604_19718_amd import binding as B
from paper_2604_19718_amd import inputs as I

pytestmark = pytest.mark.gpu

COUNT, N = 256, 64


@pytest.fixture(scope="module")
def batch():
    probs = []
    for k in range(COUNT):
        p, en = I.workload(4, index=k)
        probs.append(p)
    seed = I.sampler_seed(4)
    h = B.cdz_create(en, "fp32")
    out = B.cdz_batch(h, probs, N, seed)
    print("batch timings ms", B.cdz_last_timings(h)[:3], flush=True)
    return probs, en, seed, out


def test_lengths(batch):
    probs, en, seed, out = batch
    m = np.array([p.m for p in probs])
    assert m.min() >= 30 and m.max() <= 400 and len(set(m)) > 100


def test_members_equal_single_calls(batch):
    probs, en, seed, out = batch
    h = B.cdz_create(en, "fp32")
    m = np.array([p.m for p in probs])
    for b in (int(np.argmin(m)), int(np.argmax(m)), 17):
        r = B.cdz_marginals(h, probs[b])
        assert out["logz"][b] == r["logz"], b
        for k in ("pair", "base", "codon", "codon_pair"):
            assert np.array_equal(out[k][b], r[k]), (b, k)
        c, p = B.cdz_sample(h, probs[b], seed + b, N)
        assert np.array_equal(out["codons"][b], c) and np.array_equal(out["pairs"][b], p), b


def test_shortest_member_against_oracle(batch):
    probs, en, seed, out = batch
    b = int(np.argmin([p.m for p in probs]))
    ref = oracle.marginals(probs[b], en)
    assert abs(out["logz"][b] - ref["logz"]) <= 1e-6 * abs(ref["logz"])
    for k in ("pair", "base", "codon", "codon_pair"):
        assert np.abs(out[k][b] - ref[k]).max() <= 1e-5, k


def test_invariants_every_member(batch):
    probs, en, seed, out = batch
    for b, p in enumerate(probs):
        P = out["pair"][b]
        assert np.abs(P - P.T).max() == 0
        assert np.abs(out["base"][b].sum(1) - 1).max() < 1e-5
        assert np.abs(out["codon"][b].sum(1) - 1).max() < 1e-5
        pt = out["pairs"][b]
        assert pt.shape == (N, p.n)
        idx = np.arange(p.n)
        for s in range(0, N, 16):
            row = pt[s]
            paired = row >= 0
            assert np.all(row[row[paired]] == idx[paired])
