"""CPU emulation of the index arithmetic the diagonal kernels use to stage the
loop windows of a cell (i, j) into LDS.

The kernels read each region as contiguous row segments and place every value
into its 6 x 6 block through per-cell maps from a state offset to a position
(cdz_window_maps): mapL for positions i+1+q, mapR for positions j-1-q,
q = 0..lmax, lmax = min(30, j - i - 6).  This file restates that arithmetic
(the same formulas, written out in Python) and checks, for the cells of real
proteins, that

  * every map entry is written once and lies inside the 192-byte map;
  * every staged value lands inside its region, in the block and at the
    (row slot, column slot) of the element it was read from, and every
    element of every block the window needs is written exactly once;

for the forward window (U runs, DI strips, A of the inner cell), the outside
window (the same strips, its own DIcol offset), and both bulge strips
(left: Qb[i+1+l][j-1] from rows of Qbt; right: Qb[i+1][j-1-l] from a row of
Qb).  Proteins: the longest member of the 256-protein batch (1197 nt) and a
1300-residue protein (3900 nt).
"""
import numpy as np
import pytest

from paper_2604_19718_amd import inputs as I

MAXLOOP = 30
NA = 27
MAPSZ = 192


def _positions(prot):
    d = np.array([I.AA_DEGENERACY[ch] for ch in prot for _ in range(3)], dtype=np.int64)
    P = np.concatenate([[0], np.cumsum(d)])
    return d, P


class Cell:
    """lp_* / rp_* of the kernels: d and P of positions i+1+q and j-1-q,
    q = 0..31, zero beyond the sequence."""

    def __init__(self, d, P, i, j):
        n = len(d)
        self.i, self.j, self.n = i, j, n
        self.lmax = min(MAXLOOP, j - i - 6)
        q = np.arange(32)
        lp = i + 1 + q
        rp = j - 1 - q
        okl = (lp >= 0) & (lp < n)
        okr = (rp >= 0) & (rp < n)
        self.lp_d = np.where(okl, d[np.clip(lp, 0, n - 1)], 0)
        self.lp_P = np.where(okl, P[np.clip(lp, 0, n - 1)], 0)
        self.rp_d = np.where(okr, d[np.clip(rp, 0, n - 1)], 0)
        self.rp_P = np.where(okr, P[np.clip(rp, 0, n - 1)], 0)
        self.d1, self.dm = d[i + 1], d[j - 1]
        self.P1, self.Pm = P[i + 1], P[j - 1]
        self.maps()

    def maps(self):
        lmax = self.lmax
        mapL = -np.ones(MAPSZ, dtype=np.int64)
        mapR = -np.ones(MAPSZ, dtype=np.int64)
        for q in range(31):
            if q <= lmax:
                for c in range(self.lp_d[q]):
                    o = self.lp_P[q] - self.lp_P[0] + c
                    assert 0 <= o < MAPSZ and mapL[o] < 0
                    mapL[o] = q
                for c in range(self.rp_d[q]):
                    o = self.rp_P[q] - self.rp_P[lmax] + c
                    assert 0 <= o < MAPSZ and mapR[o] < 0
                    mapR[o] = q
        self.mapL, self.mapR = mapL, mapR


def _check_region(dest, src_row, src_col, blk_lo, nblk, want):
    """dest: LDS index of every staged value; src_row/src_col: the state
    indices it was read from (as a matrix element); want(b) -> (first row
    state, rows, first column state, columns) of block b - blk_lo.  Checks
    that each value lands in its region, inside its block's used part, at the
    slots of the element it was read from, and that every used element of
    every block is staged exactly once."""
    dest = np.asarray(dest, dtype=np.int64)
    b = dest // 36
    assert np.all((b >= blk_lo) & (b < blk_lo + nblk)), "value staged outside its region"
    spec = np.array([want(bb) for bb in range(nblk)], dtype=np.int64).reshape(nblk, 4)
    r0, nr, c0, nc = (spec[b - blk_lo, k] for k in range(4))
    rr, cc = (dest % 36) // 6, dest % 6
    assert np.all((rr < nr) & (cc < nc)), "value staged into block padding"
    assert np.all((np.asarray(src_row) == r0 + rr) & (np.asarray(src_col) == c0 + cc)), \
        "value staged at the wrong slot"
    assert np.unique(dest).size == dest.size, "two values staged to one LDS entry"
    assert dest.size == int((spec[:, 1] * spec[:, 3]).sum()), "block element never staged"


def _span(P, d, p):
    return (P[p], d[p])


def check_window(d, P, C, outside=False):
    """UR1, UC1, DIrow, DIcol (and, forward, the A blocks of the inner cell)."""
    i, j, lmax = C.i, C.j, C.lmax
    lp_P, rp_P, rp_d = C.lp_P, C.rp_P, C.rp_d
    if lmax < 1 or (outside and lmax < 2):
        return
    baseL, baseR = lp_P[0], rp_P[lmax]
    KU = lp_P[lmax] - baseL
    endR = rp_P[0] + rp_d[0] - baseR
    oC = rp_P[lmax - 1] - baseR
    KC = endR - oC
    oD = rp_P[lmax - 2] - baseR if lmax >= 2 else endR
    KD = endR - oD
    oL = lp_P[1] - baseL
    KL = lp_P[lmax - 1] - lp_P[1] if lmax >= 3 else 0
    d1, dm, P1, Pm = C.d1, C.dm, C.P1, C.Pm
    # U[i+1][i+l]: row P1 + r of U; block qq = l - 1
    idx = np.arange(d1 * KU)
    r, k = idx // max(KU, 1), idx % max(KU, 1)
    qq = C.mapL[k]
    assert np.all(qq >= 0)
    c = k - (lp_P[qq] - baseL)
    _check_region(qq * 36 + r * 6 + c, P1 + r, baseL + k, 0, lmax,
                  lambda b: (*_span(P, d, i + 1), *_span(P, d, i + 1 + b)))
    # U[j-l][j-1]: row Pm + c of Ut (element (baseR + k, Pm + c) of U); block 30 + l - 1
    t = np.arange(dm * KC)
    c, k = t // max(KC, 1), t % max(KC, 1) + oC
    qq = C.mapR[k]
    assert np.all(qq >= 0)
    r = k - (rp_P[qq] - baseR)
    _check_region((30 + qq) * 36 + r * 6 + c, baseR + k, Pm + c, 30, lmax,
                  lambda b: (*_span(P, d, j - 1 - b), *_span(P, d, j - 1)))
    # DI[i+1][j-L+1]: row P1 + r of DI; block 60 + L - 2, L = 2..lmax
    if lmax >= 2:
        t = np.arange(d1 * KD)
        r, k = t // max(KD, 1), t % max(KD, 1) + oD
        qq = C.mapR[k]
        assert np.all(qq >= 0)
        c = k - (rp_P[qq] - baseR)
        _check_region((60 + qq) * 36 + r * 6 + c, P1 + r, baseR + k, 60, lmax - 1,
                      lambda b: (*_span(P, d, i + 1), *_span(P, d, j - 1 - b)))
    # DI[i+L-1][j-1]: row Pm + c of DIt; L = 3..lmax; forward block 89 + L - 3,
    # outside block 89 + L - 2
    if lmax >= 3:
        t = np.arange(dm * KL)
        c, k = t // KL, t % KL + oL
        qq = C.mapL[k]
        assert np.all(qq >= 1)
        r = k - (lp_P[qq] - baseL)
        lo = 90 if outside else 89
        _check_region((lo - 1 + qq) * 36 + r * 6 + c, baseL + k, Pm + c, lo, lmax - 2,
                      lambda b: (*_span(P, d, i + 2 + b), *_span(P, d, j - 1)))
    # A(i+1, j-1, L), L = 2..lmax-2 (forward, all diagonals resident): rows
    # P[i+2].., columns NA * P[j-2] + (L-2) * d[j-2] + dd of the A matrix
    nAP = max(lmax - 3, 0)
    if not outside and nAP > 0:
        dA, dB = C.lp_d[1], rp_d[1]
        KA = nAP * dB
        t = np.arange(dA * KA)
        r, k = t // KA, t % KA
        dest = (117 + k // dB) * 36 + r * 6 + k % dB
        _check_region(dest, lp_P[1] + r, NA * rp_P[1] + k, 117, nAP,
                      lambda b: (*_span(P, d, i + 2), NA * P[j - 2] + b * d[j - 2], d[j - 2]))
    # the regions stay inside the window buffer: 173 blocks (forward), 118 (outside)
    assert (117 + nAP if not outside else 118) <= (173 if not outside else 118)


def check_bulges(d, P, C):
    """Left strip Qb[i+1+l][j-1] (rows of Qbt placed by mapL) and right strip
    Qb[i+1][j-1-l] (a row of Qb placed by mapR), l = 1..lmax, block l - 1."""
    i, j, lmax = C.i, C.j, C.lmax
    if lmax < 1:
        return
    lp_P, rp_P = C.lp_P, C.rp_P
    o, K = lp_P[1] - lp_P[0], lp_P[lmax + 1] - lp_P[1]
    idx = np.arange(C.dm * K)
    c, k = idx // K, idx % K + o
    l = C.mapL[k]
    assert np.all((l >= 1) & (l <= lmax))
    x = k - (lp_P[l] - lp_P[0])
    _check_region((l - 1) * 36 + x * 6 + c, lp_P[0] + k, C.Pm + c, 0, lmax,
                  lambda b: (*_span(P, d, i + 2 + b), *_span(P, d, j - 1)))
    baseR = rp_P[lmax]
    K = rp_P[1] + C.rp_d[1] - baseR  # states of positions j-1-lmax .. j-2
    idx = np.arange(C.d1 * K)
    r, k = idx // K, idx % K
    q = C.mapR[k]
    assert np.all((q >= 1) & (q <= lmax))
    c = k - (rp_P[q] - baseR)
    _check_region((q - 1) * 36 + r * 6 + c, C.P1 + r, baseR + k, 0, lmax,
                  lambda b: (*_span(P, d, i + 1), *_span(P, d, j - 2 - b)))


def _cells(n, rng, every):
    """Every cell of the diagonals with lmax < 30 (dl <= 35) at stride
    `every` in i, and on the longer diagonals one cell per i and one per j
    (the staging of a full window depends on i for the left regions and on j
    for the right ones only), plus random cells."""
    out = set()
    for dl in range(7, 36):
        for i in range(0, n - dl, every):
            out.add((i, i + dl))
    for i in range(0, n - 36):
        dl = 36 + int(rng.integers(0, n - 36 - i)) if n - 36 - i > 0 else 36
        out.add((i, i + dl))
    for j in range(36, n):
        dl = 36 + int(rng.integers(0, j - 35))
        out.add((j - dl, j))
    return sorted(out)


@pytest.mark.parametrize("which", ["batch_longest_1197nt", "workload5_3900nt"])
def test_window_staging_indices(which):
    if which == "batch_longest_1197nt":
        prob, _ = I.workload(4, index=189)
        every = 4
    else:
        prob, _ = I.workload(5)
        every = 37
    d, P = _positions(prob.prot)
    rng = np.random.default_rng(5)
    cells = _cells(len(d), rng, every)
    for (i, j) in cells:
        C = Cell(d, P, i, j)
        check_window(d, P, C, outside=False)
        check_window(d, P, C, outside=True)
        check_bulges(d, P, C)


def test_a_planted_index_mistake_is_caught():
    """The check is not vacuous: offset the right map by one state and the
    right bulge strip lands on the wrong slots."""
    prob, _ = I.workload(4, index=189)
    d, P = _positions(prob.prot)
    C = Cell(d, P, 100, 200)
    C.mapR = np.concatenate([[C.mapR[0]], C.mapR[:-1]])
    with pytest.raises(AssertionError):
        check_bulges(d, P, C)
