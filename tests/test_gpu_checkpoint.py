"""Memory-bounded form: the interior-loop sums A kept as a ring of diagonals in
the forward, checkpoints every K diagonals, and bands recomputed from them in
the outside pass.  Results must equal the all-resident form bit for bit."""
import numpy as np
import pytest
import torch

from paper_2604_19718_amd import binding as B
from paper_2604_19718_amd import inputs as I
from paper_2604_19718_amd.autograd import CdzLogZ, make_handle

pytestmark = pytest.mark.gpu

KEYS = ("pair", "base", "codon", "codon_pair")


def _al_k(h):
    return B.lib().cdz_debug_al_k(h.ptr)


def _force(h, K):
    assert B.lib().cdz_debug_force_al_k(h.ptr, K) == 0


def _equal(a, b, label):
    assert a["logz"] == b["logz"], label
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), (label, k, np.abs(a[k] - b[k]).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_budget_selects_checkpointed_form(prec):
    prob, en = I.workload(2, m=100)
    ref_h = B.cdz_create(en, prec)
    ref = B.cdz_marginals(ref_h, prob)
    assert _al_k(ref_h) == -1
    full = B.cdz_workspace_bytes(ref_h, prob, B.CDZ_WS_MARGINALS)
    low = B.cdz_workspace_bytes(ref_h, prob, B.CDZ_WS_MARGINALS_MIN)
    print(prec, "workspace", full, "checkpointed", low, flush=True)
    assert low < full
    h = B.cdz_create(en, prec, mem_budget_bytes=low)
    got = B.cdz_marginals(h, prob)
    assert _al_k(h) > 0
    _equal(got, ref, f"{prec} budget")
    # samples from the ring-form forward equal the resident form's
    a = B.cdz_sample(h, prob, 11, 16)
    b = B.cdz_sample(ref_h, prob, 11, 16)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("K", [1, 2, 3, 7, 8, 11, 16, 64, 1000])
def test_every_band_length(prec, K):
    """Band lengths around the first diagonals that read A (10 and up), one
    band covering everything, and a band longer than the sequence."""
    prob, en = I.workload(2, m=23)
    ref = B.cdz_marginals(B.cdz_create(en, prec), prob)
    h = B.cdz_create(en, prec)
    _force(h, K)
    got = B.cdz_marginals(h, prob)
    assert _al_k(h) == K
    _equal(got, ref, f"{prec} K={K}")


def test_forward_only_ring():
    prob, en = I.workload(2, m=30)
    ref_h = B.cdz_create(en, "fp32")
    lz = B.cdz_partition(ref_h, prob)
    ring = B.cdz_workspace_bytes(ref_h, prob, B.CDZ_WS_FORWARD_MIN)
    assert ring < B.cdz_workspace_bytes(ref_h, prob, B.CDZ_WS_FORWARD)
    h = B.cdz_create(en, "fp32", mem_budget_bytes=ring)
    assert B.cdz_partition(h, prob) == lz
    assert _al_k(h) == 0
    # the outside pass needs more than the ring: refused, not truncated
    assert ring < B.cdz_workspace_bytes(h, prob, B.CDZ_WS_MARGINALS_MIN)
    with pytest.raises(B.CdzError) as e:
        B.cdz_marginals(h, prob)
    assert e.value.status == 5


def test_budget_below_minimum():
    prob, en = I.workload(2, m=30)
    h0 = B.cdz_create(en, "fp32")
    low = B.cdz_workspace_bytes(h0, prob, B.CDZ_WS_MARGINALS_MIN)
    h = B.cdz_create(en, "fp32", mem_budget_bytes=low - 4096)
    with pytest.raises(B.CdzError) as e:
        B.cdz_marginals(h, prob)
    assert e.value.status == 5


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_checkpointed_gradient(prec):
    """Gradients through the torch.autograd.Function in the checkpointed form
    equal the resident form's."""
    prob, en = I.workload(2, m=50)
    outs = []
    for K in (-2, 9):
        h = make_handle(en, prec)
        _force(h, K)
        t1 = torch.tensor(prob.theta1, dtype=torch.float64, device="cuda", requires_grad=True)
        t2 = torch.tensor(prob.theta2, dtype=torch.float64, device="cuda", requires_grad=True)
        lz = CdzLogZ.apply(t1, t2, h, prob.prot)
        lz.backward()
        assert _al_k(h) == (K if K > 0 else -1)
        outs.append((lz.item(), t1.grad.cpu().numpy(), t2.grad.cpu().numpy()))
    assert outs[0][0] == outs[1][0]
    assert np.array_equal(outs[0][1], outs[1][1]) and np.array_equal(outs[0][2], outs[1][2])
