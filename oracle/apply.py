"""Operator-state multiplication from the plain definition (oracle; test use only).

A letter string acts on a computational basis state letter by letter:
X|b> = |1-b>, Y|b> = i(-1)^b |1-b>, Z|b> = (-1)^b |b>.  Hence for
P = i^gamma (x) sigma,

    P |s> = i^(gamma + #Y) (-1)^popcount(s & (Y|Z positions)) |s xor (X|Y positions)>.

H|psi> = sum_k c_k sum_s psi_s P_k|s> is evaluated term by term, scattering
from every source configuration s of the space to t = s xor flip_k
(Eq. grouped_contraction without the grouping).  In a spin sector the result
is the projection P H P psi: sources outside the sector carry no amplitude
and targets outside the sector are discarded (for a number- and
S_z-conserving H this is H psi exactly).  All arithmetic is float64.
"""

import numpy as np

from .pauli import I, X, Y, Z


def term_action(letters):
    """(flip mask, sign mask, number of Y) of letter rows [m, n] (n <= 64)."""
    letters = np.atleast_2d(np.asarray(letters, dtype=np.uint8))
    m, n = letters.shape
    assert n <= 64
    weights = np.uint64(1) << np.arange(n, dtype=np.uint64)
    flip = ((letters == X) | (letters == Y)).astype(np.uint64) @ weights
    sign = ((letters == Y) | (letters == Z)).astype(np.uint64) @ weights
    n_y = (letters == Y).sum(axis=1)
    return flip.astype(np.uint64), sign.astype(np.uint64), n_y


_IPOW = np.array([1, 1j, -1, -1j], dtype=np.complex128)


def apply_scatter(op, space, psi):
    """(P H P) psi for a letter-form PauliSum ``op`` on ``space`` (full or sector)."""
    psi = np.asarray(psi, dtype=np.complex128)
    assert psi.shape == (space.dim,)
    flip, sign, n_y = term_action(op.letters)
    src = space.basis()
    out = np.zeros(space.dim, dtype=np.complex128)
    for k in range(op.n_terms):
        tgt = space.index_of(src ^ flip[k])
        ok = tgt >= 0
        parity = np.bitwise_count(src & sign[k]) & 1
        amp = op.coeff[k] * _IPOW[n_y[k] % 4] * np.where(parity == 1, -1.0, 1.0) * psi
        out[tgt[ok]] += amp[ok]      # s -> s xor flip is injective for fixed k
    return out


def apply_targets(op, space, psi, target_index):
    """(P H P psi)[t] for selected target indices, each computed on its own:
    (H psi)_t = sum_k c_k <t|P_k|s_k> psi_{s_k} with s_k = t xor flip_k."""
    psi = np.asarray(psi)
    flip, sign, n_y = term_action(op.letters)
    factor = op.coeff * _IPOW[n_y % 4]
    basis_all = None
    out = np.zeros(len(target_index), dtype=np.complex128)
    for j, ti in enumerate(np.asarray(target_index, dtype=np.int64)):
        t = _bits_of(space, ti)
        s = t ^ flip
        si = space.index_of(s)
        ok = si >= 0
        parity = np.bitwise_count(s & sign) & 1
        vals = factor * np.where(parity == 1, -1.0, 1.0)
        out[j] = np.sum(vals[ok] * psi[si[ok]].astype(np.complex128))
    return out


def _bits_of(space, index):
    if hasattr(space, "alpha"):
        ia, ib = divmod(int(index), space.dim_beta)
        return np.uint64(int(space.alpha[ia]) | (int(space.beta[ib]) << space.n_orb))
    return np.uint64(int(index))


def expval(op, space, psi):
    """(<psi|H|psi>, <psi|psi>) in float64 (Eq. vqe_energy)."""
    psi = np.asarray(psi, dtype=np.complex128)
    hpsi = apply_scatter(op, space, psi)
    return complex(np.vdot(psi, hpsi)), float(np.vdot(psi, psi).real)


def dense_matrix(op):
    """Dense 2^n x 2^n matrix of sum_k c_k P_k (n <= 12)."""
    return op.dense()


def restrict(vec_full, space):
    """Amplitudes of a full-space vector on the configurations of ``space``."""
    return np.asarray(vec_full)[space.basis().astype(np.int64)]


def embed(vec, space, n_qubits):
    out = np.zeros(1 << n_qubits, dtype=np.complex128)
    out[space.basis().astype(np.int64)] = vec
    return out
