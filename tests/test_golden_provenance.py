"""The stored oracle values used by the full-size GPU parity tests come from
the oracle: the 300-nt file is recomputed here and must agree, and every
stored file names the oracle sources it was computed with."""
import numpy as np
import pytest

import oracle
from paper_2604_19718_amd import inputs as I

from golden.make_oracle_goldens import load, oracle_sha256


@pytest.mark.parametrize("k", [2, 3, 4])
def test_goldens_match_current_oracle_sources(k):
    assert str(load(k)["oracle_sha256"]) == oracle_sha256()


def test_300nt_golden_recomputed():
    prob, en = I.workload(2)
    ref = load(2)
    got = oracle.marginals(prob, en)
    assert abs(got["logz"] - ref["logz"]) <= 1e-13 * abs(ref["logz"])
    for key in ("pair", "base", "codon", "codon_pair"):
        assert np.abs(got[key] - ref[key]).max() <= 1e-13, key
