"""Configuration spaces and their indexing (oracle; test use only).

* Full space of n qubits: basis index = the bit pattern itself (qubit k is
  bit k of the index, Eqs. xp_encoding / zp_encoding).
* Spin sector (N_alpha, N_beta) of n_orb spatial orbitals (Section 2.4,
  spin-resolved product basis; dimension Eq. fcidim): qubits 0..n_orb-1 hold
  the alpha string, qubits n_orb..2n_orb-1 the beta string.  Each spin's
  strings are all n_orb-bit words with the required number of ones, listed in
  ascending integer order; a configuration's index is
  rank_alpha * D_beta + rank_beta (alpha-major).  The paper does not fix the
  order; ascending order with alpha outermost matches the loop nest of
  Algorithm 2 (alpha strings outer, beta strings inner).

Rank is the position in the explicitly enumerated list (binary search), not a
combinatorial formula.
"""

from itertools import combinations

import numpy as np


def spin_strings(n_orb, n_elec):
    """All n_orb-bit words with n_elec ones, ascending."""
    words = [sum(1 << i for i in c) for c in combinations(range(n_orb), n_elec)]
    return np.array(sorted(words), dtype=np.uint64)


def _find(table, values):
    values = np.asarray(values, dtype=np.uint64)
    pos = np.searchsorted(table, values)
    pos_c = np.minimum(pos, len(table) - 1)
    ok = (pos < len(table)) & (table[pos_c] == values)
    return np.where(ok, pos_c, -1).astype(np.int64)


class FullSpace:
    def __init__(self, n_qubits):
        self.n_qubits = n_qubits
        self.dim = 1 << n_qubits

    def basis(self):
        return np.arange(self.dim, dtype=np.uint64)

    def index_of(self, bits):
        bits = np.asarray(bits, dtype=np.uint64)
        return np.where(bits < np.uint64(self.dim), bits.astype(np.int64), -1)


class SectorSpace:
    def __init__(self, n_orb, n_alpha, n_beta):
        self.n_orb = n_orb
        self.n_qubits = 2 * n_orb
        self.n_alpha = n_alpha
        self.n_beta = n_beta
        self.alpha = spin_strings(n_orb, n_alpha)
        self.beta = spin_strings(n_orb, n_beta)
        self.dim_alpha = len(self.alpha)
        self.dim_beta = len(self.beta)
        self.dim = self.dim_alpha * self.dim_beta

    def basis(self):
        """Bit pattern of every configuration, in index order."""
        a = np.repeat(self.alpha, self.dim_beta)
        b = np.tile(self.beta, self.dim_alpha)
        return a | (b << np.uint64(self.n_orb))

    def index_of(self, bits):
        """Index of each bit pattern, -1 when it lies outside the sector."""
        bits = np.asarray(bits, dtype=np.uint64)
        mask = np.uint64((1 << self.n_orb) - 1)
        a = bits & mask
        b = (bits >> np.uint64(self.n_orb)) & mask
        high = bits >> np.uint64(2 * self.n_orb)
        ia = _find(self.alpha, a)
        ib = _find(self.beta, b)
        ok = (ia >= 0) & (ib >= 0) & (high == 0)
        return np.where(ok, ia * self.dim_beta + ib, -1)

    def rank_alpha(self, words):
        return _find(self.alpha, words)

    def rank_beta(self, words):
        return _find(self.beta, words)
