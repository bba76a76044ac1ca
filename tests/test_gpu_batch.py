"""Batched calls: many proteins of uneven length on one handle.

Every protein of a batch must give exactly (bit for bit) what the
single-problem calls give, whatever the chunking, and a few members are
checked against the FP64 oracle directly."""
import numpy as np
import pytest

import oracle
from paper_2604_19718_amd import binding as B
from paper_2604_19718_amd import inputs as I

pytestmark = pytest.mark.gpu

KEYS = ("pair", "base", "codon", "codon_pair")


def _members(lengths):
    """Batch members of the 256-protein workload with their lengths overridden
    (energy tables shared by the batch)."""
    out = []
    for k, m in enumerate(lengths):
        prob, en = I.workload(4, m=m, index=k)
        out.append(prob)
    return out, en


RAGGED = [1, 7, 30, 2, 19, 44, 12, 3, 33]


def _single(h, probs, seed, N):
    res = []
    for b, p in enumerate(probs):
        r = B.cdz_marginals(h, p)
        r["codons"], r["pairs"] = B.cdz_sample(h, p, seed + b, N)
        res.append(r)
    return res


def _same(batch, single):
    for b, s in enumerate(single):
        assert batch["logz"][b] == s["logz"], b
        for k in KEYS:
            assert np.array_equal(batch[k][b], s[k]), (b, k)
        assert np.array_equal(batch["codons"][b], s["codons"]), b
        assert np.array_equal(batch["pairs"][b], s["pairs"]), b


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_equals_single_calls(prec):
    probs, en = _members(RAGGED)
    seed, N = 77, 12
    h = B.cdz_create(en, prec)
    batch = B.cdz_batch(h, probs, N, seed)
    print("batch", prec, [round(x, 6) for x in batch["logz"]], flush=True)
    _same(batch, _single(B.cdz_create(en, prec), probs, seed, N))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_chunked_by_budget(prec):
    """A budget that holds only a few proteins at a time: several chunks, the
    same outputs as one chunk."""
    probs, en = _members(RAGGED)
    seed, N = 5, 4
    h0 = B.cdz_create(en, prec)
    whole = B.cdz_batch(h0, probs, N, seed)
    need = [B.cdz_workspace_bytes(h0, p, B.CDZ_WS_MARGINALS) for p in probs]
    budget = max(need) + min(need)
    chunks, used = 1, 0
    for x in need:
        if used + x > budget:
            chunks, used = chunks + 1, 0
        used += x
    assert chunks >= 3
    part = B.cdz_batch(B.cdz_create(en, prec, mem_budget_bytes=budget), probs, N, seed)
    for k in ("logz",):
        assert np.array_equal(whole[k], part[k])
    for k in KEYS + ("codons", "pairs"):
        for b in range(len(probs)):
            assert np.array_equal(whole[k][b], part[k][b]), (k, b)


def test_batch_budget_below_one_protein():
    probs, en = _members([20, 5])
    h = B.cdz_create(en, "fp32", mem_budget_bytes=1 << 20)
    with pytest.raises(B.CdzError) as e:
        B.cdz_batch(h, probs, 0, 0)
    assert e.value.status == 5  # CDZ_ERR_BUDGET


def test_batch_reports_bad_member_index():
    probs, en = _members([4, 4])
    probs[1] = I.Problem("MKXL", None, None)
    h = B.cdz_create(en, "fp32")
    with pytest.raises(B.CdzError) as e:
        B.cdz_partition_batch(h, probs)
    assert e.value.status == 2 and "problem 1" in str(e.value)


def test_batch_empty():
    _, en = _members([3])
    h = B.cdz_create(en, "fp32")
    assert B.cdz_partition_batch(h, []).shape == (0,)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_members_against_oracle(prec):
    probs, en = _members([9, 26, 2, 15])
    got = B.cdz_marginals_batch(B.cdz_create(en, prec), probs)
    atol = 1e-10 if prec == "fp64" else 1e-5
    rtol = 1e-12 if prec == "fp64" else 1e-6
    for b, p in enumerate(probs):
        ref = oracle.marginals(p, en)
        assert abs(got["logz"][b] - ref["logz"]) <= rtol * max(1, abs(ref["logz"])), b
        for k in KEYS:
            err = np.abs(got[k][b] - ref[k]).max()
            print(prec, b, k, f"{err:.3e}", flush=True)
            assert err <= atol, (b, k, err)


def test_batch_after_single_call_recomputes():
    """A batch overwrites the workspace: a following single-problem sample must
    recompute its forward and still equal a fresh handle's."""
    probs, en = _members([10, 6])
    h = B.cdz_create(en, "fp32")
    B.cdz_partition(h, probs[0])
    B.cdz_partition_batch(h, probs)
    a = B.cdz_sample(h, probs[0], 3, 8)
    b = B.cdz_sample(B.cdz_create(en, "fp32"), probs[0], 3, 8)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
