"""GPU forward pass (log Z) against the FP64 oracle, through the C ABI."""
import math

import numpy as np
import pytest

import oracle
from paper_2604_19718_amd import binding as B
from paper_2604_19718_amd import inputs as I

pytestmark = pytest.mark.gpu

# tolerances of the two precision modes (relative, on log Z)
TOL = {"fp64": 1e-12, "fp32": 1e-6}


def _rel(a, b):
    return abs(a - b) / max(1.0, abs(b))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("prot", ["M", "KW", "KLV", "MKWLRS", "GASCYHWQ"])
def test_small_proteins(prec, prot):
    en = I.energy_tables(1001)
    prob = I.Problem(prot, I.theta1(5, prot), I.theta2(5, prot))
    ref = oracle.logz(prob, en)
    h = B.cdz_create(en, prec)
    got = B.cdz_partition(h, prob)
    print(prec, prot, got, ref, flush=True)
    assert _rel(got, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_workload_8aa(prec):
    prob, en = I.workload(1)
    ref = oracle.logz(prob, en)
    got = B.cdz_partition(B.cdz_create(en, prec), prob)
    assert _rel(got, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("m", [17, 45, 100])
def test_workload_300nt(prec, m):
    prob, en = I.workload(2, m=m)
    ref = oracle.logz(prob, en)
    h = B.cdz_create(en, prec)
    got = B.cdz_partition(h, prob)
    suffix = B.lib().cdz_debug_logz_suffix(h.ptr)
    print(prec, m, got, suffix, ref, got - ref, flush=True)
    assert _rel(got, ref) <= TOL[prec]
    assert _rel(suffix, ref) <= TOL[prec]
