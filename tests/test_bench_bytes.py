"""The algorithmic byte counts bench.py prices its rooflines with, against a
per-cell loop over the same definition (split stream or pulls plus the blocks
a cell writes; padding never counts)."""
import numpy as np
import pytest

import bench


def _loop_fwd(d, w):
    n = len(d)
    P = np.concatenate([[0], np.cumsum(d)])
    tot = 0
    for i in range(n):
        for j in range(i + 4, n):
            K = P[j - 4] - P[i + 4] if j - i >= 9 else 0
            tot += (d[i] + d[j]) * K + 5 * d[i] * d[j]
    return tot * w


def _loop_out(d, w):
    n = len(d)
    P = np.concatenate([[0], np.cumsum(d)])
    tot = 0
    for i in range(n):
        for j in range(i, n):
            own = d[i] * d[j]
            if j - i < 4:
                tot += 7 * own
                continue
            KR = P[n] - P[j + 5] if j + 5 <= n - 1 else 0
            KL = P[i - 4] if i >= 5 else 0
            dim1 = d[i - 1] if i >= 1 else 0
            djp1 = d[j + 1] if j + 1 <= n - 1 else 0
            tot += (d[i] + d[j]) * KR + (dim1 + d[j]) * KL
            tot += 7 * own + dim1 * d[j] + dim1 * djp1 + 2 * d[i + 1] * d[j - 1]
    return tot * w


@pytest.mark.parametrize("n,seed", [(4, 0), (9, 1), (23, 2), (40, 3)])
def test_byte_counts_match_cell_loop(n, seed):
    d = np.random.default_rng(seed).integers(1, 7, size=n).astype(np.int64)
    assert bench.algorithmic_bytes_fwd(d, 4) == _loop_fwd(d, 4)
    assert bench.algorithmic_bytes_out(d, 4) == _loop_out(d, 4)
    assert bench.algorithmic_bytes_out(d, 8) == _loop_out(d, 8)


def _loop_tensor(sig, g, elt):
    """Row by row: each row r of position block p < j reads Q[r][off[p] .. off[j]),
    the fold row block j (g Sigma_j rows of off[j]) is read once and the column
    (off[j] rows of g Sigma_j) written once; flops 2 g Sigma_j per element read."""
    n = len(sig) - 1
    off = [0]
    for p in range(n + 1):
        off.append(off[-1] + g * int(sig[p]))
    tb = tf = 0
    for j in range(1, n + 1):
        R, w = off[j], g * int(sig[j])
        tri = 0
        for p in range(j):
            for r in range(off[p], off[p + 1]):
                tri += R - off[p]
        tb += (tri + 2 * w * R) * elt
        tf += 2 * tri * w
    return tb, tf


@pytest.mark.parametrize("prot,g", [("M", 9), ("MKWLRS", 9), ("ACDEFGHIKLMNPQRSTVWY", 4)])
def test_tensor_bytes(prot, g):
    from paper_2604_19718_amd import binding as B
    from paper_2604_19718_amd import inputs as I
    sig = B.cdz_tensor_dims(I.Problem(prot, None, None))
    assert bench.tensor_prop_algorithmic(sig, g, 4) == _loop_tensor(sig, g, 4)


def test_tensor_dims_match_the_oracle():
    """The library's single-codon train dimensions (host only, no device) against
    the oracle's, for every amino acid."""
    import oracle
    from paper_2604_19718_amd import binding as B
    from paper_2604_19718_amd import inputs as I
    prot = I.AA_ORDER + "MWLSRKV"
    assert np.array_equal(B.cdz_tensor_dims(I.Problem(prot, None, None)), oracle.tensor_dims(prot))
