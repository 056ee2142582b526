"""Pauli strings and Pauli sums from their definitions (oracle; test use only).

A string is kept as a row of letters (0 = I, 1 = X, 2 = Y, 3 = Z), qubit k in
column k, with a global phase i^gamma, gamma in Z4 ("letter form"): the
operator is i^gamma (x) sigma_k.  The binary symplectic pair of a string is
read off the letters with the bit-pair convention of Eq. single_pauli_mapping
(I = (0,0), X = (1,0), Y = (1,1), Z = (0,1)), packed as in Eqs.
xp_encoding/zp_encoding into 64-bit words (word w holds qubits 64w..64w+63).

Readings of the paper used here:
* Eq. pauli_group states gamma in {0,1}; products generate all four powers
  of i, so gamma is read as an element of Z4.
* A Pauli sum is stored with letter-form coefficients c_j (the operator is
  sum_j c_j (x) sigma), so a Hermitian sum has real coefficients.  The paper's
  C_j = c_j * Lambda_j (Section 2.3) is the same sum written against
  X^x Z^z, which the kernels use internally.
* Canonical form (Section 2.3): unique strings ordered by (X, Z) read as
  unsigned big integers, X major; each coefficient is the correctly rounded
  exact sum of its contributions (real and imaginary parts separately, an
  exact zero written as +0.0); a term is dropped when max(|Re c|, |Im c|) <=
  eps_drop.  The paper fixes neither the summation order nor the norm of the
  drop test; exact rounding makes the result independent of input order.
"""

import math
from dataclasses import dataclass

import numpy as np

I, X, Y, Z = 0, 1, 2, 3
_LETTER = "IXYZ"


def _letter_tables():
    """sigma_a sigma_b = delta_ab I + i eps_abc sigma_c for a, b in {X, Y, Z};
    I is the identity of the product.  Returns (letter, phase exponent)."""
    prod = np.zeros((4, 4), dtype=np.uint8)
    phase = np.zeros((4, 4), dtype=np.uint8)
    cyclic = {(X, Y): Z, (Y, Z): X, (Z, X): Y}
    for a in range(4):
        for b in range(4):
            if a == I:
                prod[a, b] = b
            elif b == I:
                prod[a, b] = a
            elif a == b:
                prod[a, b] = I
            elif (a, b) in cyclic:
                prod[a, b] = cyclic[(a, b)]
                phase[a, b] = 1          # +i
            else:
                prod[a, b] = cyclic[(b, a)]
                phase[a, b] = 3          # -i
    return prod, phase


LETTER_PRODUCT, LETTER_PHASE = _letter_tables()

_SIGMA = [
    np.array([[1, 0], [0, 1]], dtype=np.complex128),
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
]
I_POW = np.array([1, 1j, -1, -1j], dtype=np.complex128)


def parse(text):
    """'XIZY' (qubit 0 first) -> uint8 letter row."""
    return np.array([_LETTER.index(ch) for ch in text], dtype=np.uint8)


def to_text(row):
    return "".join(_LETTER[int(v)] for v in row)


def string_product(la, pa, lb, pb):
    """Product (i^pa A)(i^pb B) of letter strings, qubit by qubit.

    la, lb: uint8 [..., n]; pa, pb: Z4 exponents [...]; returns (letters, phase)."""
    la = np.asarray(la, dtype=np.uint8)
    lb = np.asarray(lb, dtype=np.uint8)
    letters = LETTER_PRODUCT[la, lb]
    extra = LETTER_PHASE[la, lb].astype(np.int64).sum(axis=-1)
    phase = (np.asarray(pa, dtype=np.int64) + np.asarray(pb, dtype=np.int64) + extra) % 4
    return letters, phase.astype(np.uint8)


def n_words(n_qubits):
    return max(1, (n_qubits + 63) // 64)


def letters_to_xz(letters):
    """Letter rows [m, n] -> (x, z) uint64 words [m, W] (Eq. single_pauli_mapping,
    Eqs. xp_encoding / zp_encoding)."""
    letters = np.atleast_2d(np.asarray(letters, dtype=np.uint8))
    m, n = letters.shape
    w = n_words(n)
    xbit = (letters == X) | (letters == Y)
    zbit = (letters == Y) | (letters == Z)
    x = np.zeros((m, w), dtype=np.uint64)
    z = np.zeros((m, w), dtype=np.uint64)
    for k in range(n):
        word, bit = divmod(k, 64)
        one = np.uint64(1) << np.uint64(bit)
        x[:, word] |= np.where(xbit[:, k], one, np.uint64(0))
        z[:, word] |= np.where(zbit[:, k], one, np.uint64(0))
    return x, z


def xz_to_letters(x, z, n_qubits):
    """Inverse of letters_to_xz: (1,1) -> Y, (1,0) -> X, (0,1) -> Z."""
    x = np.atleast_2d(np.asarray(x, dtype=np.uint64))
    z = np.atleast_2d(np.asarray(z, dtype=np.uint64))
    m = x.shape[0]
    out = np.zeros((m, n_qubits), dtype=np.uint8)
    for k in range(n_qubits):
        word, bit = divmod(k, 64)
        xb = (x[:, word] >> np.uint64(bit)) & np.uint64(1)
        zb = (z[:, word] >> np.uint64(bit)) & np.uint64(1)
        out[:, k] = np.where(xb & zb, Y, np.where(xb, X, np.where(zb, Z, I)))
    return out


def dense_string(letters, phase=0):
    """Dense 2^n x 2^n matrix of i^phase (x) sigma with qubit k = bit k of the
    basis index (qubit 0 is the rightmost Kronecker factor)."""
    mat = np.array([[1.0 + 0j]])
    for letter in letters[::-1]:
        mat = np.kron(mat, _SIGMA[int(letter)])
    return I_POW[int(phase) % 4] * mat


@dataclass
class PauliSum:
    """sum_j coeff[j] * (x) sigma(letters[j])  (letter-form coefficients)."""

    n_qubits: int
    letters: np.ndarray   # uint8 [m, n]
    coeff: np.ndarray     # complex128 [m]

    @property
    def n_terms(self):
        return int(self.coeff.shape[0])

    def xz(self):
        return letters_to_xz(self.letters.reshape(-1, self.n_qubits))

    def dense(self):
        dim = 1 << self.n_qubits
        out = np.zeros((dim, dim), dtype=np.complex128)
        for row, c in zip(self.letters, self.coeff):
            out += c * dense_string(row)
        return out

    @staticmethod
    def from_text(terms, n_qubits=None):
        """[(text, coeff), ...] -> PauliSum (not canonicalised)."""
        if n_qubits is None:
            n_qubits = len(terms[0][0])
        letters = np.array([parse(t) for t, _ in terms], dtype=np.uint8).reshape(-1, n_qubits)
        coeff = np.array([complex(c) for _, c in terms], dtype=np.complex128)
        return PauliSum(n_qubits, letters, coeff)

    def as_dict(self):
        return {to_text(r): complex(c) for r, c in zip(self.letters, self.coeff)}


def sum_product(a, b):
    """(sum_k a_k P_k)(sum_l b_l Q_l) = sum_kl a_k b_l P_k Q_l, every pair kept
    (Eq. pauli_operator_multiplication before reduction)."""
    assert a.n_qubits == b.n_qubits
    ka = np.repeat(np.arange(a.n_terms), b.n_terms)
    kb = np.tile(np.arange(b.n_terms), a.n_terms)
    letters, phase = string_product(a.letters[ka], 0, b.letters[kb], 0)
    coeff = a.coeff[ka] * b.coeff[kb] * I_POW[phase]
    return PauliSum(a.n_qubits, letters, coeff)


def sum_product_canonical(a, b, eps_drop=0.0):
    """Canonical form of (sum_k a_k P_k)(sum_l b_l Q_l) with every coefficient
    the correctly rounded value of its exact sum (Eq.
    pauli_operator_multiplication followed by the canonical reduction of
    Section 2.3).  Pair products are accumulated as exact rationals and
    rounded once."""
    from fractions import Fraction

    assert a.n_qubits == b.n_qubits
    acc = {}
    for k in range(a.n_terms):
        letters, phase = string_product(a.letters[k][None, :].repeat(b.n_terms, 0), 0, b.letters, 0)
        px, pz = letters_to_xz(letters)
        ar, ai = Fraction(a.coeff[k].real), Fraction(a.coeff[k].imag)
        for l in range(b.n_terms):
            br, bi = Fraction(b.coeff[l].real), Fraction(b.coeff[l].imag)
            re, im = ar * br - ai * bi, ar * bi + ai * br
            for _ in range(int(phase[l])):           # multiply by i
                re, im = -im, re
            key = (tuple(int(v) for v in px[l][::-1]), tuple(int(v) for v in pz[l][::-1]))
            if key in acc:
                acc[key][0] += re
                acc[key][1] += im
            else:
                acc[key] = [re, im]
    keys = sorted(acc)
    w = n_words(a.n_qubits)
    xs = np.array([list(k[0][::-1]) for k in keys], dtype=np.uint64).reshape(-1, w)
    zs = np.array([list(k[1][::-1]) for k in keys], dtype=np.uint64).reshape(-1, w)
    re = np.array([float(acc[k][0]) + 0.0 for k in keys])
    im = np.array([float(acc[k][1]) + 0.0 for k in keys])
    keep = np.maximum(np.abs(re), np.abs(im)) > eps_drop
    return xs[keep], zs[keep], (re + 1j * im)[keep]


def sort_order(x, z):
    """Permutation ordering keys by (X, Z) as big unsigned integers, X major."""
    w = x.shape[1]
    keys = [z[:, i] for i in range(w)] + [x[:, i] for i in range(w)]
    return np.lexsort(keys)


def _exact_sum(values):
    s = math.fsum(values)
    return s + 0.0  # exact zero is written as +0.0


def canonicalize_xz(x, z, re, im, eps_drop=0.0):
    """Canonical reduction on symplectic keys (Section 2.3).

    x, z: uint64 [m, W]; re, im: float64 [m] (letter-form coefficient parts).
    Returns (x, z, coeff) with unique sorted keys, correctly rounded sums and
    the drop rule max(|re|, |im|) <= eps_drop."""
    x = np.asarray(x, dtype=np.uint64).reshape(len(re), -1)
    z = np.asarray(z, dtype=np.uint64).reshape(len(re), -1)
    re = np.asarray(re, dtype=np.float64)
    im = np.asarray(im, dtype=np.float64)
    if len(re) == 0:
        return x[:0], z[:0], np.zeros(0, np.complex128)
    order = sort_order(x, z)
    xs, zs, rs, is_ = x[order], z[order], re[order], im[order]
    key = np.concatenate([xs, zs], axis=1)
    head = np.ones(len(rs), dtype=bool)
    head[1:] = np.any(key[1:] != key[:-1], axis=1)
    starts = np.flatnonzero(head)
    ends = np.append(starts[1:], len(rs))
    out_re = np.empty(len(starts))
    out_im = np.empty(len(starts))
    rl, il = rs.tolist(), is_.tolist()
    for g, (s, e) in enumerate(zip(starts.tolist(), ends.tolist())):
        out_re[g] = _exact_sum(rl[s:e])
        out_im[g] = _exact_sum(il[s:e])
    keep = np.maximum(np.abs(out_re), np.abs(out_im)) > eps_drop
    coeff = out_re + 1j * out_im
    return xs[starts][keep], zs[starts][keep], coeff[keep]


def canonicalize(s, eps_drop=0.0):
    """PauliSum -> canonical PauliSum (letters rebuilt from the sorted keys)."""
    x, z = s.xz()
    xo, zo, c = canonicalize_xz(x, z, s.coeff.real, s.coeff.imag, eps_drop)
    return PauliSum(s.n_qubits, xz_to_letters(xo, zo, s.n_qubits), c)


def canonical_arrays(s, eps_drop=0.0):
    """PauliSum -> (x [m,W], z [m,W], coeff [m]) in canonical form."""
    x, z = s.xz()
    return canonicalize_xz(x, z, s.coeff.real, s.coeff.imag, eps_drop)


def commutes(la, lb):
    """True when two letter strings commute: they anticommute on an odd number
    of positions where both are non-identity and different."""
    la = np.asarray(la)
    lb = np.asarray(lb)
    anti = (la != I) & (lb != I) & (la != lb)
    return int(anti.sum()) % 2 == 0


def group_by_x(x, z, coeff):
    """Partition canonical terms by X-mask (Eq. topological_group).

    Returns (xg [G], offsets [G+1], z [M], C [M]) where C_k = c_k * Lambda_k
    with Lambda_k = i^popcount(X_k & Z_k) (Section 2.3), i.e. the coefficient
    of X^x Z^z.  Groups appear in the canonical order (ascending X); exact
    zeros are written as +0.0, as in the canonical form."""
    x = np.asarray(x, dtype=np.uint64).reshape(len(coeff), -1)
    z = np.asarray(z, dtype=np.uint64).reshape(len(coeff), -1)
    assert x.shape[1] == 1, "single-word masks only"
    xs = x[:, 0]
    heads = np.ones(len(xs), dtype=bool)
    heads[1:] = xs[1:] != xs[:-1]
    starts = np.flatnonzero(heads)
    offsets = np.append(starts, len(xs)).astype(np.uint64)
    n_y = np.bitwise_count(xs & z[:, 0]).astype(np.int64)
    lam = I_POW[n_y % 4]
    return xs[starts], offsets, z[:, 0].copy(), np.asarray(coeff) * lam + 0.0
