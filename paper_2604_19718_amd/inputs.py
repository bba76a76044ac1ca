"""Seeded synthetic inputs for the codon-constrained partition function.

This module only draws random numbers and lays them out as arrays: it holds
none of the method's arithmetic (no Boltzmann factors, no recursions, no
codon spelling).  Both the HIP path and the CPU oracle take their inputs from
here, so a parity test compares the two on identical bytes.

Workload recipe (stand-in for the paper's random-protein benchmark of the
scaling study in Section 5b and the SI; the paper draws amino acids with the
Spike composition and uses a trained tensor model, neither of which is
available, so amino acids are uniform and the energy tables synthetic):

* amino acids uniform over the 20 standard letters, order ``ARNDCQEGHILKMFPSTWYV``;
* nearest-neighbour tables in kT with Turner-like magnitudes (see
  :func:`energy_tables`);
* codon weights: log w ~ N(0, 0.5^2) per sense-codon type, codon-pair weights
  log w ~ N(0, 0.3^2) per ordered pair of sense-codon types, both expanded to
  the protein's positions (the soft constraints of Section 3a).

Tensor-model workload (Sections 3b-3c; the paper's trained (nu=3, mu=3,
xi=1) parameters are not available, so V, B and S are synthetic with the same
shapes: gamma = nu * mu = 9, rank xi = 1; see :func:`tensor_model`).

Random streams: SplitMix64 sub-streams keyed by (master seed, tag, index) with
tags 0 protein, 1 energy tables, 2 codon weights, 3 codon-pair weights,
4 sampler key, 5 finite-difference index choice, 6 tensor-model parameters.  Uniforms take the top 53
bits; Gaussians use Box-Muller.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np

AA_ORDER = "ARNDCQEGHILKMFPSTWYV"
# Number of sense codons per amino acid (standard genetic code), in AA_ORDER.
# Codon *types* are the pairs (amino acid, slot) for slot < count; the
# spelling of each slot is not needed to draw weights.
AA_DEGENERACY = dict(zip(AA_ORDER, [4, 6, 2, 2, 2, 2, 2, 4, 2, 3,
                                    6, 2, 1, 2, 4, 6, 4, 1, 2, 4]))
MAX_SLOTS = 6

TAG_PROTEIN, TAG_ENERGY, TAG_THETA1, TAG_THETA2, TAG_SAMPLER, TAG_FD, TAG_TENSOR = range(7)
_MASK64 = (1 << 64) - 1


def _splitmix64(state: int) -> tuple[int, int]:
    state = (state + 0x9E3779B97F4A7C15) & _MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return state, z ^ (z >> 31)


class Stream:
    """SplitMix64 sub-stream for (seed, tag, index)."""

    def __init__(self, seed: int, tag: int, index: int = 0):
        st, a = _splitmix64(seed & _MASK64)
        st, b = _splitmix64((a ^ (tag * 0xD1B54A32D192ED03)) & _MASK64)
        _, c = _splitmix64((b ^ (index * 0x8CB92BA72F3D8DD7)) & _MASK64)
        self.state = c

    def u64(self) -> int:
        self.state, z = _splitmix64(self.state)
        return z

    def uniform(self) -> float:
        """Uniform on [0, 1) with 53 random bits."""
        return (self.u64() >> 11) * (1.0 / 9007199254740992.0)

    def uniform_ab(self, a: float, b: float) -> float:
        return a + (b - a) * self.uniform()

    def gauss(self, sigma: float = 1.0) -> float:
        u1 = self.uniform()
        u2 = self.uniform()
        return sigma * math.sqrt(-2.0 * math.log(1.0 - u1)) * math.cos(2.0 * math.pi * u2)

    def randint(self, n: int) -> int:
        return int(self.uniform() * n)


@dataclass
class Energy:
    """Nearest-neighbour loop tables in kT (+inf marks a forbidden entry).

    Pair types are AU=0, CG=1, GC=2, UA=3, GU=4, UG=5; bases A=0, C=1, G=2,
    U=3.  ``mismatch[x][y][t]``: x is the base after the 5' base of the
    closing pair inside the loop, y the base before its 3' base, t the pair
    type read in loop order.
    """
    stack: np.ndarray      # [6][6]
    hairpin: np.ndarray    # [31]
    bulge: np.ndarray      # [31]
    interior: np.ndarray   # [31]
    mismatch: np.ndarray   # [4][4][6]
    ml_a: float
    ml_b: float
    ml_c: float
    extrap: float = 1.75

    def packed(self) -> np.ndarray:
        """Flat float64 record in the field order of the C-ABI energy struct."""
        return np.concatenate([
            self.stack.reshape(-1), self.hairpin, self.bulge, self.interior,
            self.mismatch.reshape(-1),
            np.array([self.ml_a, self.ml_b, self.ml_c, self.extrap]),
        ]).astype(np.float64)

    PACKED_LEN = 36 + 31 * 3 + 96 + 4

    def copy(self) -> "Energy":
        return Energy(self.stack.copy(), self.hairpin.copy(), self.bulge.copy(),
                      self.interior.copy(), self.mismatch.copy(),
                      self.ml_a, self.ml_b, self.ml_c, self.extrap)


def energy_tables(seed: int, index: int = 0) -> Energy:
    """Synthetic nearest-neighbour tables, drawn in a fixed order."""
    r = Stream(seed, TAG_ENERGY, index)
    inf = math.inf
    stack = np.array([[r.uniform_ab(-5.5, -1.5) for _ in range(6)] for _ in range(6)])
    hairpin = np.full(31, inf)
    for L in range(3, 31):
        hairpin[L] = 8.5 + 1.75 * math.log(L / 3.0) + r.uniform_ab(-0.5, 0.5)
    bulge = np.full(31, inf)
    for L in range(1, 31):
        bulge[L] = 6.0 + 1.75 * math.log(L) + r.uniform_ab(-0.5, 0.5)
    interior = np.full(31, inf)
    for L in range(2, 31):
        interior[L] = 1.5 + 1.75 * math.log(L / 2.0) + r.uniform_ab(-0.5, 0.5)
    mismatch = np.array([[[r.uniform_ab(-2.5, 0.0) for _ in range(6)]
                          for _ in range(4)] for _ in range(4)])
    ml_a = r.uniform_ab(4.5, 6.5)
    ml_b = r.uniform_ab(0.0, 0.8)
    ml_c = r.uniform_ab(0.0, 0.3)
    return Energy(stack, hairpin, bulge, interior, mismatch, ml_a, ml_b, ml_c, 1.75)


def zero_energy() -> Energy:
    """All loop energies zero (every structure weighs 1), minimum sizes kept."""
    e = energy_tables(0)
    inf = math.inf
    e.stack[:] = 0.0
    e.hairpin[:] = [inf if L < 3 else 0.0 for L in range(31)]
    e.bulge[:] = [inf if L < 1 else 0.0 for L in range(31)]
    e.interior[:] = [inf if L < 2 else 0.0 for L in range(31)]
    e.mismatch[:] = 0.0
    e.ml_a = e.ml_b = e.ml_c = 0.0
    e.extrap = 0.0
    return e


def hairpin_only_energy(seed: int) -> Energy:
    """The synthetic tables with every loop except hairpins forbidden: every
    structure is a set of side-by-side hairpins in the exterior loop, so long
    hairpins carry a visible share of Z (a test model)."""
    e = energy_tables(seed)
    e.stack[:] = math.inf
    e.bulge[:] = math.inf
    e.interior[:] = math.inf
    e.ml_a = math.inf
    return e


def interior_rich_energy(seed: int) -> Energy:
    """Stacks and bulges forbidden, interior loops favourable and strongly
    mismatch-dependent, so that helices are built from interior loops (a test
    model for the interior-loop terms)."""
    e = energy_tables(seed)
    r = Stream(seed, TAG_ENERGY, 99)
    e.stack[:] = math.inf
    e.bulge[:] = math.inf
    for L in range(2, 31):
        e.interior[L] = -2.0 + 0.1 * L
    e.mismatch[:] = np.array([[[r.uniform_ab(-4.0, 0.0) for _ in range(6)]
                               for _ in range(4)] for _ in range(4)])
    e.hairpin[3:] = e.hairpin[3:] - 3.0
    return e


def bulge_rich_energy(seed: int) -> Energy:
    """Stacks and interior loops forbidden, bulges favourable and more so the
    longer they are, so that helices are built from bulges and the longest
    bulges carry a visible share of Z (a test model for the bulge terms)."""
    e = energy_tables(seed)
    e.stack[:] = math.inf
    e.interior[:] = math.inf
    for L in range(1, 31):
        e.bulge[L] = -1.0 - 0.1 * L
    e.hairpin[3:] = e.hairpin[3:] - 3.0
    return e


def protein(seed: int, m: int, index: int = 0) -> str:
    r = Stream(seed, TAG_PROTEIN, index)
    return "".join(AA_ORDER[r.randint(20)] for _ in range(m))


def _codon_types():
    return [(a, s) for a in AA_ORDER for s in range(AA_DEGENERACY[a])]


def theta1(seed: int, prot: str, sigma: float = 0.5, index: int = 0) -> np.ndarray:
    """Position-level log codon weights [m][6] from one weight per codon type."""
    r = Stream(seed, TAG_THETA1, index)
    typ = {t: r.gauss(sigma) for t in _codon_types()}
    out = np.zeros((len(prot), MAX_SLOTS))
    for a, ch in enumerate(prot):
        for s in range(AA_DEGENERACY[ch]):
            out[a, s] = typ[(ch, s)]
    return out


def bonus_targets(seed: int, sigma: float = 0.5, index: int = 0) -> np.ndarray:
    """Target codon bonuses [26][6] (row = letter - 'A', column = slot): the
    per-codon-type weights theta1 draws, exponentiated, so that theta1 of any
    protein under the same seed is log of these at its residues' codons."""
    r = Stream(seed, TAG_THETA1, index)
    out = np.zeros((26, MAX_SLOTS))
    for (a, s) in _codon_types():
        out[ord(a) - 65, s] = math.exp(r.gauss(sigma))
    return out


def theta2(seed: int, prot: str, sigma: float = 0.3, index: int = 0) -> np.ndarray:
    """Position-level log codon-pair weights [m][6][6]; row a couples codon
    a-1 (first index) with codon a (second index); row 0 is zero."""
    r = Stream(seed, TAG_THETA2, index)
    types = _codon_types()
    tab = np.array([[r.gauss(sigma) for _ in types] for _ in types])
    pos = {t: k for k, t in enumerate(types)}
    out = np.zeros((len(prot), MAX_SLOTS, MAX_SLOTS))
    for a in range(1, len(prot)):
        p, c = prot[a - 1], prot[a]
        for s in range(AA_DEGENERACY[p]):
            for t in range(AA_DEGENERACY[c]):
                out[a, s, t] = tab[pos[(p, s)], pos[(c, t)]]
    return out


@dataclass
class Problem:
    prot: str
    theta1: Optional[np.ndarray]
    theta2: Optional[np.ndarray]

    @property
    def m(self) -> int:
        return len(self.prot)

    @property
    def n(self) -> int:
        return 3 * len(self.prot)


def config_seed(k: int) -> int:
    return 1000 + k


def workload(k: int, m: Optional[int] = None, index: int = 0):
    """(Problem, Energy) for the numbered workload k.

    1: 8 aa, codon weights only; 2: 100 aa, codon + pair weights;
    3: 300 aa (900 nt), codon + pair weights; 4: batch member ``index`` with
    m ~ U{30..400}; 5: 1300 aa.  ``m`` overrides the length.
    """
    seed = config_seed(k)
    if m is None:
        if k == 4:
            m = 30 + Stream(seed, TAG_PROTEIN, 10_000 + index).randint(371)
        else:
            m = {1: 8, 2: 100, 3: 300, 5: 1300}[k]
    prot = protein(seed, m, index)
    en = energy_tables(seed)
    t1 = theta1(seed, prot, 0.5, index)
    t2 = None if k == 1 else theta2(seed, prot, 0.3, index)
    return Problem(prot, t1, t2), en


def sampler_seed(k: int, index: int = 0) -> int:
    return Stream(config_seed(k), TAG_SAMPLER, index).u64()


# ---- tensor-based structure model (synthetic parameters) -------------------

PAIRABLE = {(0, 3): 1.0, (3, 0): 1.0, (1, 2): 1.6, (2, 1): 1.6, (2, 3): 0.6, (3, 2): 0.6}


@dataclass
class TensorModel:
    """Parameters of a tensor-based secondary-structure model: V[4][g][g]
    per unpaired base, B[xi][4][4][g][g] per side of a pair (first index the
    base of that side, second its partner; zero for bases that do not pair),
    S[g][g] for the weighted trace.  Bases A=0, C=1, G=2, U=3."""
    V: np.ndarray
    B: np.ndarray
    S: np.ndarray

    @property
    def gamma(self) -> int:
        return self.V.shape[1]

    @property
    def xi(self) -> int:
        return self.B.shape[0]


def tensor_model(seed: int, gamma: int = 9, xi: int = 1, pair: float = 1.0, index: int = 0) -> TensorModel:
    """Synthetic non-negative parameters with the trained model's shapes.

    V_b: entries U(0.2, 1), each row then divided by its sum (row-stochastic,
    so spectral radius 1, the normalisation the paper applies to its V).
    B_{x,y}: for the six pairing combinations (AU, UA, CG, GC, GU, UG),
    entries U(0, 1) * strength(x, y) * pair / gamma (GC 1.6, AU 1.0, GU 0.6);
    zero otherwise.  S: entries U(0.5, 1.5) / gamma."""
    r = Stream(seed, TAG_TENSOR, index)
    V = np.array([[[r.uniform_ab(0.2, 1.0) for _ in range(gamma)] for _ in range(gamma)] for _ in range(4)])
    V /= V.sum(axis=2, keepdims=True)
    B = np.zeros((xi, 4, 4, gamma, gamma))
    for rho in range(xi):
        for (x, y), st in PAIRABLE.items():
            B[rho, x, y] = np.array([[r.uniform() * st * pair / gamma for _ in range(gamma)]
                                     for _ in range(gamma)])
    S = np.array([[r.uniform_ab(0.5, 1.5) / gamma for _ in range(gamma)] for _ in range(gamma)])
    return TensorModel(V, B, S)


def tensor_workload(k: int, m: Optional[int] = None):
    """(Problem, TensorModel) for the tensor-model workload k: the protein and
    codon bonuses of workload k (no codon-pair weights: the single-codon
    tensor train carries per-codon bonuses only) and synthetic (9, 1) model
    parameters."""
    prob, _ = workload(k, m)
    return Problem(prob.prot, prob.theta1, None), tensor_model(config_seed(k))
