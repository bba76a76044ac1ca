"""Error paths of the boundary (inputs are validated before any device work)
and run-to-run determinism of the kernels."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2604_19718_amd import binding as B
from paper_2604_19718_amd import inputs as I

pytestmark = pytest.mark.gpu

ARG, PROTEIN, NUMERIC, STATE = 1, 2, 3, 7


def _status(fn):
    with pytest.raises(B.CdzError) as e:
        fn()
    return e.value.status


def test_bad_inputs():
    prob, en = I.workload(1)
    h = B.cdz_create(en, "fp32")
    assert _status(lambda: B.cdz_partition(h, I.Problem("MK*V", None, None))) == PROTEIN
    assert _status(lambda: B.cdz_partition(h, I.Problem("MKBV", None, None))) == PROTEIN
    assert _status(lambda: B.cdz_partition(h, I.Problem("", None, None))) == ARG
    t1 = prob.theta1.copy()
    t1[2, 0] = np.nan
    assert _status(lambda: B.cdz_partition(h, I.Problem(prob.prot, t1, None))) == NUMERIC
    t1[2, 0] = np.inf
    assert _status(lambda: B.cdz_partition(h, I.Problem(prob.prot, t1, None))) == NUMERIC
    t1[2, 0] = -np.inf
    assert _status(lambda: B.cdz_partition(h, I.Problem(prob.prot, t1, None))) == NUMERIC
    pp = B._Prob(prob)
    assert B.lib().cdz_sample(h.ptr, ctypes.byref(pp.c), 1, -1, None, None) == ARG
    # the handle still works after rejected calls
    assert abs(B.cdz_partition(h, prob) - oracle.logz(prob, en)) <= 1e-6 * 20


def test_bad_energy_tables():
    _, en = I.workload(1)
    bad = en.copy()
    bad.stack[0, 0] = np.nan
    assert _status(lambda: B.cdz_create(bad, "fp32")) == NUMERIC
    bad = en.copy()
    bad.hairpin[5] = -np.inf
    assert _status(lambda: B.cdz_create(bad, "fp64")) == NUMERIC


def test_backward_without_forward():
    import torch
    _, en = I.workload(1)
    h = B.cdz_create(en, "fp64")
    g1 = torch.zeros((8, 6), dtype=torch.float64, device="cuda")
    assert B.lib().cdz_backward_dev(h.ptr, 1.0, ctypes.c_void_p(g1.data_ptr()), None) == STATE
    assert B.lib().cdz_backward_dev(h.ptr, 1.0, None, None) == ARG


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["300nt", "1197nt"])
def test_runs_are_bitwise_repeatable(prec, case):
    if case == "300nt":
        prob, en = I.workload(2)
    else:
        prob, en = I.workload(4, index=189)
        assert prob.n == 1197
    outs = [B.cdz_marginals(B.cdz_create(en, prec), prob) for _ in range(2)]
    assert outs[0]["logz"] == outs[1]["logz"]
    for k in ("pair", "base", "codon", "codon_pair"):
        assert np.array_equal(outs[0][k], outs[1][k]), k
