"""GPU outside pass (adjoint) and marginals against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_2604_19718_amd import binding as B
from paper_2604_19718_amd import inputs as I

pytestmark = pytest.mark.gpu

# absolute tolerance on marginals (probabilities) per precision mode
ATOL = {"fp64": 1e-10, "fp32": 1e-5}
KEYS = ("pair", "base", "codon", "codon_pair")


def _check(got, ref, prec, label):
    assert abs(got["logz"] - ref["logz"]) <= (1e-12 if prec == "fp64" else 1e-6) * max(1, abs(ref["logz"]))
    for k in KEYS:
        err = np.abs(got[k] - ref[k]).max()
        print(label, prec, k, f"{err:.3e}", flush=True)
        assert err <= ATOL[prec], (k, err)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("prot", ["M", "KW", "KLV", "MKWLRS", "GASCYHWQ"])
def test_small(prec, prot):
    en = I.energy_tables(1001)
    prob = I.Problem(prot, I.theta1(5, prot), I.theta2(5, prot))
    ref = oracle.marginals(prob, en)
    got = B.cdz_marginals(B.cdz_create(en, prec), prob)
    _check(got, ref, prec, prot)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_workload_8aa(prec):
    prob, en = I.workload(1)
    ref = oracle.marginals(prob, en)
    got = B.cdz_marginals(B.cdz_create(en, prec), prob)
    _check(got, ref, prec, "w1")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("m", [23, 60])
def test_workload_ragged(prec, m):
    prob, en = I.workload(2, m=m)
    ref = oracle.marginals(prob, en)
    got = B.cdz_marginals(B.cdz_create(en, prec), prob)
    _check(got, ref, prec, f"m{m}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("model", ["bulge_rich", "interior_rich"])
def test_loop_rich_models(prec, model):
    """Tables under which bulges and interior loops up to the 30-nt window
    limit carry a visible share of Z, so that a dropped or misplaced long-loop
    term moves the marginals far beyond the tolerance."""
    en = getattr(I, f"{model}_energy")(7)
    prob, _ = I.workload(2, m=40)
    ref = oracle.marginals(prob, en)
    got = B.cdz_marginals(B.cdz_create(en, prec), prob)
    _check(got, ref, prec, model)
