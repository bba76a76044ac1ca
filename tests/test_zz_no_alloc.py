"""cdz_sample_noalloc, the sampler entry point that allocates no device
memory (its workspace is a fixed per-device array), called through the C ABI:
its samples equal cdz_sample's bit for bit on two calls in a row, the second
with a smaller input; requests beyond its scratch and calls without the
problem's forward pass are refused."""
import numpy as np
import pytest

from paper_2604_19718_amd import binding as B
from paper_2604_19718_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_sampler_equals_cdz_sample(prec):
    big, en = I.workload(3)       # 900 nt, 1000 samples (30.8 MB of scratch)
    small, _ = I.workload(2)      # then 300 nt, 100 samples, on the same scratch
    h = B.cdz_create(en, prec)
    for prob, N, seed in ((big, 1000, I.sampler_seed(3)), (small, 100, I.sampler_seed(2))):
        B.cdz_partition(h, prob)
        c0, p0 = B.cdz_sample_noalloc(h, prob, seed, N)
        c1, p1 = B.cdz_sample(h, prob, seed, N)
        print(prec, prob.n, N, "codon mismatches", int((c0 != c1).sum()), "pair mismatches",
              int((p0 != p1).sum()), flush=True)
        assert np.array_equal(c0, c1) and np.array_equal(p0, p1)
    # again after a regular call reused the handle's own workspace
    c2, p2 = B.cdz_sample_noalloc(h, small, 11, 7)
    c3, p3 = B.cdz_sample(h, small, 11, 7)
    assert np.array_equal(c2, c3) and np.array_equal(p2, p3)


def test_noalloc_refusals():
    big, en = I.workload(3)
    small, _ = I.workload(2)
    h = B.cdz_create(en, "fp32")
    with pytest.raises(B.CdzError) as e:          # no forward pass in the handle
        B.cdz_sample_noalloc(h, small, 1, 4)
    assert e.value.status == 7
    B.cdz_partition(h, big)
    with pytest.raises(B.CdzError) as e:          # another problem's forward pass
        B.cdz_sample_noalloc(h, small, 1, 4)
    assert e.value.status == 7
    with pytest.raises(B.CdzError) as e:          # beyond the 32 MiB scratch
        B.cdz_sample_noalloc(h, big, 1, 2000)
    assert e.value.status == 5 and "scratch" in str(e.value)
    c, p = B.cdz_sample_noalloc(h, big, 1, 0)
    assert c.shape == (0, big.m)
