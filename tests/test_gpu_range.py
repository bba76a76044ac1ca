"""The floating-point range machinery of the forward pass.

FP32 keeps every diagonal within range by an exact power-of-two landscape
rescaling estimated from a span-truncated pass; after the exact pass a range
check flags cells whose largest entry fell below 2^-e (zero included) and
non-finite entries.  A weak pass is repeated once with the landscape of the
exact pass; still weak, or non-finite, the call returns CDZ_ERR_NUMERIC.
These tests force both branches through the test hooks of
include/cdz_debug.h (a poor landscape estimate from span-4 truncation, a
raised threshold) in the single and the batched calls, and run tables far
outside the synthetic ranges, which must give the oracle's values or
CDZ_ERR_NUMERIC, never wrong numbers."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2604_19718_amd import binding as B
from paper_2604_19718_amd import inputs as I

from golden.make_oracle_goldens import load as load_golden

pytestmark = pytest.mark.gpu


def _hooked(en, span, low):
    h = B.cdz_create(en, "fp32")
    assert B.lib().cdz_debug_set_span(h.ptr, span) == 0
    assert B.lib().cdz_debug_set_low_exp(h.ptr, low) == 0
    return h


def _weakest(h):
    f, g = ctypes.c_int(), ctypes.c_int()
    assert B.lib().cdz_debug_weakest(h.ptr, ctypes.byref(f), ctypes.byref(g)) == 0
    return f.value, g.value


def _spread(prob, en, span):
    """Binary exponent of the weakest cell after the exact pass and after the
    repeated one, found with a threshold no cell meets (2^-1): the call must
    repeat the pass and then fail with CDZ_ERR_NUMERIC."""
    h = _hooked(en, span, 1)
    with pytest.raises(B.CdzError) as e:
        B.cdz_partition(h, prob)
    assert e.value.status == 3  # CDZ_ERR_NUMERIC
    assert B.lib().cdz_debug_landscape_retries(h.ptr) == 1
    return _weakest(h)


def _between(first, final):
    """A threshold exponent that the exact pass fails and the repeated pass meets."""
    assert final > first + 1, (first, final)
    return (-first - final) // 2


@pytest.fixture(scope="module")
def spread900():
    prob, en = I.workload(3)
    first, final = _spread(prob, en, 4)
    print("900 nt, span-4 landscape: weakest cell 2^%d, after the repeated pass 2^%d" % (first, final), flush=True)
    return prob, en, first, final


def test_repeated_pass_900nt_matches_oracle(spread900):
    """Span-4 truncation (no pair fits) gives a poor landscape estimate, so the
    cells of the exact pass spread further than those of the repeated pass,
    whose landscape comes from the exact pass.  With a threshold between the
    two spreads the pass is repeated once and then clears the check; log Z
    and marginals still match the oracle."""
    prob, en, first, final = spread900
    ref = load_golden(3)
    h = _hooked(en, 4, _between(first, final))
    m = B.cdz_marginals(h, prob)
    assert B.lib().cdz_debug_landscape_retries(h.ptr) == 1
    assert abs(m["logz"] - ref["logz"]) <= 1e-6 * abs(ref["logz"])
    for key in ("pair", "base", "codon", "codon_pair"):
        assert np.abs(m[key] - ref[key]).max() <= 1e-5, key


def test_repeated_pass_300nt_matches_oracle():
    prob, en = I.workload(2)
    ref = load_golden(2)
    first, final = _spread(prob, en, 4)
    h = _hooked(en, 4, _between(first, final))
    m = B.cdz_marginals(h, prob)
    assert B.lib().cdz_debug_landscape_retries(h.ptr) == 1
    assert abs(m["logz"] - ref["logz"]) <= 1e-6 * abs(ref["logz"])
    for key in ("pair", "codon"):
        assert np.abs(m[key] - ref[key]).max() <= 1e-5, key


def test_still_weak_after_repeat_is_an_error():
    """A threshold just above the weakest cell of the repeated pass: the pass
    is repeated, still fails the check, and the call returns CDZ_ERR_NUMERIC
    (partition and marginals alike)."""
    prob, en = I.workload(2)
    first, final = _spread(prob, en, 0)
    h = _hooked(en, 0, max(1, -final - 3))
    with pytest.raises(B.CdzError) as e:
        B.cdz_partition(h, prob)
    assert e.value.status == 3
    assert B.lib().cdz_debug_landscape_retries(h.ptr) == 1
    with pytest.raises(B.CdzError) as e:
        B.cdz_marginals(h, prob)
    assert e.value.status == 3


def test_batched_repeat_and_error(spread900):
    """The batched call takes the same branches per member: a repeated pass
    that clears the check gives the single call's values bit for bit; a
    member still weak after the repeat fails the call with CDZ_ERR_NUMERIC."""
    prob, en, first, final = spread900
    small = I.Problem("MKVLAW", None, None)
    ref = load_golden(3)
    low = _between(first, final)
    h = _hooked(en, 4, low)
    got = B.cdz_partition_batch(h, [prob, small])
    assert B.lib().cdz_debug_landscape_retries(h.ptr) >= 1
    assert abs(got[0] - ref["logz"]) <= 1e-6 * abs(ref["logz"])
    hs = _hooked(en, 4, low)
    assert got[0] == B.cdz_partition(hs, prob)
    hb = _hooked(en, 4, 1)
    with pytest.raises(B.CdzError) as e:
        B.cdz_partition_batch(hb, [small, prob])
    assert e.value.status == 3


@pytest.fixture(scope="module")
def extreme():
    """Stacking free energies of -20 kT on every pair type (the synthetic
    tables draw them in [-5.5, -1.5]): Z spans thousands of nats over 300 nt
    and strong and weak windows differ by far more than FP32 can hold."""
    prob, en = I.workload(2)
    e2 = en.copy()
    e2.stack[:] = -20.0
    return prob, e2, oracle.marginals(prob, e2)


def test_extreme_tables_fp64_matches_oracle(extreme):
    prob, e2, ref = extreme
    h = B.cdz_create(e2, "fp64")
    m = B.cdz_marginals(h, prob)
    print("fp64", m["logz"], ref["logz"], flush=True)
    assert abs(m["logz"] - ref["logz"]) <= 1e-12 * abs(ref["logz"])
    for key in ("pair", "base", "codon", "codon_pair"):
        assert np.abs(m[key] - ref[key]).max() <= 1e-10, key


def test_extreme_tables_fp32_oracle_or_error(extreme):
    prob, e2, ref = extreme
    h = B.cdz_create(e2, "fp32")
    try:
        m = B.cdz_marginals(h, prob)
    except B.CdzError as e:
        assert e.status == 3
        print("fp32:", e, flush=True)
        return
    assert abs(m["logz"] - ref["logz"]) <= 1e-6 * abs(ref["logz"])
    for key in ("pair", "codon"):
        assert np.abs(m[key] - ref[key]).max() <= 1e-5, key
