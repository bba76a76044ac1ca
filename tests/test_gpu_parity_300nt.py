"""The 300-nt workload (100 residues, codon + codon-pair weights): log Z and
all four marginals element by element against the FP64 oracle in both
precisions, and log Z of the longest batch member (1197 nt) against the
oracle.  The oracle values are stored by tests/golden/make_oracle_goldens.py,
which calls only the oracle."""
import numpy as np
import pytest

from paper_2604_19718_amd import binding as B
from paper_2604_19718_amd import inputs as I

from golden.make_oracle_goldens import BATCH_LONGEST
from golden.make_oracle_goldens import load as load_golden

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-12, 1e-10), "fp32": (1e-6, 1e-5)}


@pytest.fixture(scope="module")
def w2():
    prob, en = I.workload(2)
    ref = load_golden(2)
    assert int(ref["n"]) == prob.n
    out = {}
    for prec in ("fp64", "fp32"):
        h = B.cdz_create(en, prec)
        out[prec] = (h, B.cdz_marginals(h, prob))
    return prob, ref, out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_logz_300nt(w2, prec):
    prob, ref, out = w2
    h, mm = out[prec]
    tl, _ = TOL[prec]
    suffix = B.lib().cdz_debug_logz_suffix(h.ptr)
    print(prec, mm["logz"], suffix, ref["logz"], flush=True)
    assert abs(mm["logz"] - ref["logz"]) <= tl * abs(ref["logz"])
    assert abs(suffix - ref["logz"]) <= tl * abs(ref["logz"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("key", ["pair", "base", "codon", "codon_pair"])
def test_marginals_300nt(w2, prec, key):
    prob, ref, out = w2
    _, mm = out[prec]
    _, ta = TOL[prec]
    err = np.abs(mm[key] - ref[key])
    print(prec, key, "max abs err", err.max(), flush=True)
    assert err.max() <= ta


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_logz_1197nt(prec):
    prob, en = I.workload(4, index=BATCH_LONGEST)
    ref = load_golden(4)
    assert int(ref["n"]) == prob.n == 1197
    got = B.cdz_partition(B.cdz_create(en, prec), prob)
    tl, _ = TOL[prec]
    print(prec, got, ref["logz"], flush=True)
    assert abs(got - ref["logz"]) <= tl * abs(ref["logz"])
