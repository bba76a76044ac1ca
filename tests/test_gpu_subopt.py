"""Suboptimal states within an energy gap of the minimum (SI S4d) through
the C-ABI, against the oracle (oracle/mfe.c ``orc_subopt``).

Both sides run the same depth-first search over the argmin traceback's
decisions and evaluate every alternative with the same FP64 additions as the
forward pass, so the states, their order and their energies agree exactly
(1e-12 relative is asked of the energies); the set itself is pinned to brute
force by tests/test_oracle_subopt.py."""
import numpy as np
import pytest

import oracle
from paper_2604_19718_amd import binding as B
from paper_2604_19718_amd import inputs as I

pytestmark = pytest.mark.gpu


def _multiloop_energy():
    en = I.energy_tables(1001).copy()
    en.ml_a, en.ml_b = -15.0, -2.0
    en.hairpin[:] = [x - 6.0 for x in en.hairpin]
    return en


def _energy(kind):
    return {"default": I.energy_tables(1001), "multiloop": _multiloop_energy(),
            "interior": I.interior_rich_energy(7), "bulge": I.bulge_rich_energy(7)}[kind]


def _compare(prob, en, gap, max_states):
    ref = oracle.subopt(prob, en, gap, max_states=max_states)
    h = B.cdz_create(en, "fp32")  # the search runs in FP64 whatever the handle's precision
    got = B.cdz_subopt(h, prob, gap, max_states=max_states)
    print(prob.prot[:12], gap, "states", len(got[1]), "oracle", len(ref[1]), flush=True)
    assert abs(got[0] - ref[0]) <= 1e-12 * max(1.0, abs(ref[0]))
    assert got[4] == ref[4]
    assert len(got[1]) == len(ref[1])
    assert np.all(np.abs(got[1] - ref[1]) <= 1e-12 * np.maximum(1.0, np.abs(ref[1])))
    assert np.array_equal(got[2], ref[2]) and np.array_equal(got[3], ref[3])
    return got


CASES = [("GCAR", "default", 1.5), ("VVVP", "multiloop", 4.0), ("CYHW", "interior", 5.0),
         ("MKWL", "bulge", 6.0), ("M", "default", 2.0), ("CYHW", "default", 0.0)]


@pytest.mark.parametrize("prot,kind,gap", CASES)
def test_subopt_against_oracle_small(prot, kind, gap):
    prob = I.Problem(prot, I.theta1(5, prot, 0.5), I.theta2(5, prot, 0.3))
    _compare(prob, _energy(kind), gap, 5000)


def test_subopt_every_state():
    """An unbounded gap: the whole ensemble of a 4-residue protein, in order."""
    prob = I.Problem("GCAR", I.theta1(5, "GCAR", 0.5), I.theta2(5, "GCAR", 0.3))
    got = _compare(prob, _energy("default"), 1e6, 10000)
    assert len(got[1]) == 8056


@pytest.mark.parametrize("m,gap", [(30, 1.0), (60, 0.5), (100, 0.3)])
def test_subopt_against_oracle_larger(m, gap):
    prob, en = I.workload(2, m=m)
    _compare(prob, en, gap, 20000)


def test_subopt_limit_and_errors():
    prob, en = I.workload(2, m=30)
    got = _compare(prob, en, 1.0, 3)
    assert not got[4] and len(got[1]) == 3
    h = B.cdz_create(en, "fp64")
    for gap in (-1.0, float("nan"), float("inf")):
        with pytest.raises(B.CdzError) as e:
            B.cdz_subopt(h, prob, gap)
        assert e.value.status == 1
    # the handle still works afterwards, and the minimum agrees with cdz_mfe
    v, _, _ = B.cdz_mfe(h, prob)
    assert v == B.cdz_subopt(h, prob, 0.0, 10)[0]
