"""Batched chunks run as captured hipGraphs: the forward passes up to the range
check and the outside pass of a chunk are captured the first time its launch
sequence is seen and replayed when it recurs.  Every replay must give exactly
(bit for bit) what direct launches give, also with other work of the program
and synchronisations between the replays; a changed batch is captured anew."""
import numpy as np
import pytest

from paper_2604_19718_amd import binding as B
from paper_2604_19718_amd import inputs as I

pytestmark = pytest.mark.gpu

KEYS = ("logz", "pair", "base", "codon", "codon_pair")


def _members(lengths, first=0):
    out = []
    for k, m in enumerate(lengths):
        prob, en = I.workload(4, m=m, index=first + k)
        out.append(prob)
    return out, en


def _counts(h):
    import ctypes
    c, r = ctypes.c_int(0), ctypes.c_int(0)
    assert B.lib().cdz_debug_graph_counts(h.ptr, ctypes.byref(c), ctypes.byref(r)) == 0
    return c.value, r.value


def _same(a, b):
    for k in KEYS:
        if k == "logz":
            assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
        else:
            for x, y in zip(a[k], b[k]):
                assert np.array_equal(x, y), k


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_replays_equal_direct_launches(prec):
    probs, en = _members([5, 31, 12, 44, 2, 20])
    other, _ = _members([17], first=50)
    h = B.cdz_create(en, prec)
    B.lib().cdz_debug_set_graphs(h.ptr, 0)
    ref = B.cdz_marginals_batch(h, probs)
    assert _counts(h) == (0, 0)
    B.lib().cdz_debug_set_graphs(h.ptr, 1)
    got = B.cdz_marginals_batch(h, probs)
    print(prec, "first call: captures, replays", _counts(h), flush=True)
    assert _counts(h) == (2, 0)  # forward and outside of the one chunk
    _same(got, ref)
    for rep in range(3):
        # the program's own eager work between replays
        B.cdz_marginals(h, other[0])
        got = B.cdz_marginals_batch(h, probs)
        print(prec, "replay", rep, _counts(h), flush=True)
        assert _counts(h) == (0, 2)
        _same(got, ref)
    # another batch: captured anew, then the first one replays still
    probs2, _ = _members([9, 26, 3])
    B.lib().cdz_debug_set_graphs(h.ptr, 0)
    ref2 = B.cdz_marginals_batch(h, probs2)
    B.lib().cdz_debug_set_graphs(h.ptr, 1)
    got2 = B.cdz_marginals_batch(h, probs2)
    assert _counts(h)[0] == 2
    _same(got2, ref2)


def test_chunked_batch_graphs():
    """A budget that splits the batch into chunks: one pair of graphs per chunk."""
    probs, en = _members([40, 38, 35, 30, 25, 44])
    h0 = B.cdz_create(en, "fp32")
    B.lib().cdz_debug_set_graphs(h0.ptr, 0)
    ref = B.cdz_marginals_batch(h0, probs)
    need = 0
    for p in probs:
        need = max(need, B.cdz_workspace_bytes(h0, p, B.CDZ_WS_MARGINALS))
    h = B.cdz_create(en, "fp32", mem_budget_bytes=int(2.2 * need))
    got = B.cdz_marginals_batch(h, probs)
    c, r = _counts(h)
    print("chunked: captures, replays", c, r, flush=True)
    assert c >= 4 and r == 0
    _same(got, ref)
    got = B.cdz_marginals_batch(h, probs)
    c2, r2 = _counts(h)
    # chunks of equal images replay; the cache holds the most recent graphs
    assert c2 + r2 == c
    _same(got, ref)
