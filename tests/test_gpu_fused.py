"""Launch grouping of the diagonal kernels: every launch fused (one workgroup
per cell index running every kind of work in turn), every launch split (one
workgroup per piece of work) and the mixed default give the same results bit
for bit, single problems and batches, both precisions."""
import numpy as np
import pytest

from paper_2604_19718_amd import binding as B
from paper_2604_19718_amd import inputs as I

pytestmark = pytest.mark.gpu

KEYS = ("pair", "base", "codon", "codon_pair")
NEVER = 1 << 30


def _run_single(h, prob, fuse):
    assert B.lib().cdz_debug_set_fuse(h.ptr, fuse) == 0
    B.cdz_reset(h)
    r = B.cdz_marginals(h, prob)
    r["codons"], r["pairs"] = B.cdz_sample(h, prob, 123, 50)
    return r


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("m", [1, 8, 33, 100])
def test_single_fused_equals_split(prec, m):
    prob, en = I.workload(2, m=m)
    h = B.cdz_create(en, prec)
    ref = _run_single(h, prob, NEVER)
    for fuse in (0, 2000):
        got = _run_single(h, prob, fuse)
        print(prec, m, fuse, got["logz"], ref["logz"], flush=True)
        assert got["logz"] == ref["logz"]
        for k in KEYS + ("codons", "pairs"):
            assert np.array_equal(got[k], ref[k]), k


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_fused_equals_split(prec):
    probs = [I.workload(4, m=mm, index=k)[0] for k, mm in enumerate([3, 40, 17, 61, 9])]
    en = I.workload(4, index=0)[1]
    h = B.cdz_create(en, prec)
    out = {}
    for fuse in (NEVER, 0, 3000):
        assert B.lib().cdz_debug_set_fuse(h.ptr, fuse) == 0
        out[fuse] = B.cdz_marginals_batch(h, probs)
    for fuse in (0, 3000):
        assert np.array_equal(np.asarray(out[fuse]["logz"]), np.asarray(out[NEVER]["logz"]))
        for k in KEYS:
            for x, y in zip(out[fuse][k], out[NEVER][k]):
                assert np.array_equal(x, y), (fuse, k)


def test_fuse_hook_rejects_negative():
    prob, en = I.workload(1)
    h = B.cdz_create(en, "fp32")
    assert B.lib().cdz_debug_set_fuse(h.ptr, -2) == 1
    assert B.lib().cdz_debug_set_fuse(h.ptr, -1) == 0


def test_tuner_passes_give_identical_results():
    """The tuner's trial passes (one untimed, three candidate thresholds) and
    the settled choice all give the same bits; the batch is big enough that
    the candidates group its early launches differently."""
    probs = [I.workload(4, m=60, index=k)[0] for k in range(40)]
    en = I.workload(4, index=0)[1]
    h = B.cdz_create(en, "fp32")
    assert B.lib().cdz_debug_set_fuse(h.ptr, -1) == 0
    ref = B.cdz_marginals_batch(h, probs)
    for rep in range(4):
        got = B.cdz_marginals_batch(h, probs)
        assert np.array_equal(np.asarray(got["logz"]), np.asarray(ref["logz"])), rep
        for k in KEYS:
            for x, y in zip(got[k], ref[k]):
                assert np.array_equal(x, y), (rep, k)
