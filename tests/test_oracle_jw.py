"""Pins of the oracle's Jordan-Wigner Hamiltonian: the ladder strings, the
canonical anticommutation relations, number and hopping operators in closed
form, a dense fermionic Hamiltonian built from the occupation-number
definition of a+/a, Hermiticity, closed-form term counts and Slater-Condon
matrix elements."""

from itertools import product
from math import comb

import numpy as np
import pytest

import synth
from oracle import apply as oapply
from oracle import jw, pauli, space
from oracle.pauli import PauliSum
from tests.conftest import golden_rows


def _dict(x, z, c, n):
    return {pauli.to_text(r): v for r, v in zip(pauli.xz_to_letters(x, z, n), c)}


def test_ladder_golden():
    want = {}
    for op, p, text, re, im in golden_rows("jw_ladder_n4.txt"):
        want.setdefault((op, int(p)), {})[text] = complex(float(re), float(im))
    for (op, p), terms in want.items():
        got = jw.ladder_sum(4, p, op == "create").as_dict()
        assert got == terms


def _anticomm(a, b):
    n = a.n_qubits
    ab = pauli.sum_product(a, b)
    ba = pauli.sum_product(b, a)
    both = PauliSum(n, np.concatenate([ab.letters, ba.letters]), np.concatenate([ab.coeff, ba.coeff]))
    x, z, c = pauli.canonical_arrays(both)
    return _dict(x, z, c, n)


def test_canonical_anticommutation_exact():
    n = 5
    ident = "I" * n
    for p in range(n):
        for q in range(n):
            ann_p = jw.ladder_sum(n, p, False)
            cre_q = jw.ladder_sum(n, q, True)
            d = _anticomm(ann_p, cre_q)
            assert d == ({ident: 1.0 + 0j} if p == q else {})
            d2 = _anticomm(jw.ladder_sum(n, p, False), jw.ladder_sum(n, q, False))
            assert d2 == {}


def test_number_operator_closed_form():
    n = 4
    for p in range(n):
        h1 = np.zeros((n, n))
        h1[p, p] = 1.0
        x, z, c = jw.jw_hamiltonian(h1, np.zeros((n,) * 4))
        zp = ["I"] * n
        zp[p] = "Z"
        assert _dict(x, z, c, n) == {"I" * n: 0.5 + 0j, "".join(zp): -0.5 + 0j}


def test_hopping_closed_form():
    # a+_p a_q + a+_q a_p = 1/2 (X_p Z..Z X_q + Y_p Z..Z Y_q), p < q
    n = 6
    for p, q in [(0, 1), (1, 4), (0, 5)]:
        h1 = np.zeros((n, n))
        h1[p, q] = h1[q, p] = 1.0
        x, z, c = jw.jw_hamiltonian(h1, np.zeros((n,) * 4))
        xx = ["I"] * n
        yy = ["I"] * n
        for k in range(p + 1, q):
            xx[k] = yy[k] = "Z"
        xx[p], xx[q], yy[p], yy[q] = "X", "X", "Y", "Y"
        assert _dict(x, z, c, n) == {"".join(xx): 0.5 + 0j, "".join(yy): 0.5 + 0j}


def _fermion_dense(h1, h2, e0):
    """H in the occupation-number basis from the definition of a+ and a:
    a+_p|n> = (-1)^(sum_{k<p} n_k) |n + e_p> if n_p = 0, else 0 (bit k of the
    basis index is the occupation of mode k)."""
    n = h1.shape[0]
    dim = 1 << n

    def create(p):
        m = np.zeros((dim, dim))
        for s in range(dim):
            if not (s >> p) & 1:
                sign = (-1) ** bin(s & ((1 << p) - 1)).count("1")
                m[s | (1 << p), s] = sign
        return m

    cre = [create(p) for p in range(n)]
    ann = [c.T for c in cre]
    H = e0 * np.eye(dim)
    for p, q in product(range(n), repeat=2):
        if h1[p, q] != 0:
            H = H + h1[p, q] * cre[p] @ ann[q]
    for p, q, r, s in product(range(n), repeat=4):
        if h2[p, q, r, s] != 0:
            H = H + 0.5 * h2[p, q, r, s] * cre[p] @ cre[q] @ ann[r] @ ann[s]
    return H


@pytest.mark.parametrize("n", [3, 4, 6])
def test_dense_fermionic_hamiltonian(n):
    # general (non-symmetric, complex-free) spin-orbital tensors, plus e0
    rng = np.random.default_rng(100 + n)
    h1 = rng.standard_normal((n, n))
    h2 = rng.standard_normal((n,) * 4) * (rng.random((n,) * 4) < 0.5)
    e0 = 0.75
    x, z, c = jw.jw_hamiltonian(h1, h2, e0)
    H = PauliSum(n, pauli.xz_to_letters(x, z, n), c)
    np.testing.assert_allclose(H.dense(), _fermion_dense(h1, h2, e0), atol=1e-12)


def test_dense_molecular_hamiltonian_and_trace():
    h1, h2 = synth.molecular_spin_integrals(3, seed=7)
    x, z, c = jw.jw_hamiltonian(h1, h2, 0.0)
    n = 6
    H = PauliSum(n, pauli.xz_to_letters(x, z, n), c)
    dense = H.dense()
    np.testing.assert_allclose(dense, _fermion_dense(h1, h2, 0.0), atol=1e-12)
    # Tr(H) / 2^n is the identity coefficient
    ident = np.flatnonzero((x[:, 0] == 0) & (z[:, 0] == 0))
    assert abs(np.trace(dense) / 2 ** n - c[ident[0]]) < 1e-12


def _closed_counts(n_o):
    m = 1 + 2 * n_o + comb(2 * n_o, 2) + 4 * comb(n_o, 2) * (2 * n_o - 1) + 12 * comb(n_o, 4) + 4 * comb(n_o, 2) ** 2
    g = 1 + 2 * comb(n_o, 2) + 2 * comb(n_o, 4) + comb(n_o, 2) ** 2
    return m, g


@pytest.mark.parametrize("n_o", [2, 3, 4, 5, 6])
def test_counts_and_hermiticity(n_o):
    h1, h2 = synth.molecular_spin_integrals(n_o, seed=1000 + n_o)
    x, z, c = jw.jw_hamiltonian(h1, h2)
    m, g = _closed_counts(n_o)
    assert len(c) == m
    assert len(np.unique(x[:, 0])) == g
    # Hermitian H with real integrals: letter-form coefficients are real,
    # and the exact reduction makes every imaginary part exactly +0.0
    assert (c.imag == 0).all()
    assert not np.signbit(c.imag).any()


def test_eps_threshold_strict():
    n = 4
    h1 = np.zeros((n, n))
    h1[0, 1] = h1[1, 0] = 1e-3
    h1[2, 2] = 0.5
    x, z, c = jw.jw_hamiltonian(h1, np.zeros((n,) * 4), eps=1e-3)
    d = _dict(x, z, c, n)
    assert d == {"IIII": 0.25 + 0j, "IIZI": -0.25 + 0j}


def _apply_fermion_string(ops, occ, n):
    """Apply a product of ladder operators (rightmost first) to basis bits occ."""
    sign = 1
    for p, dagger in reversed(ops):
        bit = (occ >> p) & 1
        if dagger == bool(bit):
            return 0, 0
        sign *= (-1) ** bin(occ & ((1 << p) - 1)).count("1")
        occ ^= 1 << p
    return sign, occ


def _fermion_element(h1, h2, t, s, n):
    """<t|H|s> from the occupation-number definition of a+/a (brute force
    over the integrals that can connect s to t)."""
    val = 0.0
    for p, q in zip(*np.nonzero(h1)):
        sg, occ = _apply_fermion_string([(p, True), (q, False)], s, n)
        if sg and occ == t:
            val += sg * h1[p, q]
    diff = s ^ t
    for P, Q, R, S in zip(*np.nonzero(h2)):
        touched = (1 << int(P)) | (1 << int(Q)) | (1 << int(R)) | (1 << int(S))
        if diff & ~touched:
            continue
        sg, occ = _apply_fermion_string([(P, True), (Q, True), (R, False), (S, False)], s, n)
        if sg and occ == t:
            val += 0.5 * sg * h2[P, Q, R, S]
    return val


def test_slater_condon_elements_20_qubits():
    n_o = 10
    h, g = synth.molecular_integrals(n_o, seed=3)
    h1, h2 = synth.spin_orbital_integrals(h, g)
    op = jw.jw_sum(h1, h2)
    sp = space.SectorSpace(n_o, 5, 5)
    # Hartree-Fock determinant: lowest 5 alpha and 5 beta orbitals
    hf = (1 << 5) - 1
    hf_bits = hf | (hf << n_o)
    occ = list(range(5))
    # closed form: sum_P h_PP + 1/2 sum_PQ [(PP|QQ) - delta_spin (PQ|QP)]
    e_hf = 2 * sum(h[i, i] for i in occ)
    e_hf += 0.5 * sum(4 * g[i, i, j, j] - 2 * g[i, j, j, i] for i in occ for j in occ)
    rng = np.random.default_rng(5)
    targets = [hf_bits,
               hf_bits ^ (1 << 4) ^ (1 << 7),                              # alpha single
               hf_bits ^ (1 << 4) ^ (1 << 8) ^ (1 << (n_o + 3)) ^ (1 << (n_o + 9)),  # alpha-beta double
               hf_bits ^ (1 << 3) ^ (1 << 4) ^ (1 << 6) ^ (1 << 9)]        # alpha-alpha double
    for t in targets:
        ti = int(sp.index_of(np.array([t], np.uint64))[0])
        si = int(sp.index_of(np.array([hf_bits], np.uint64))[0])
        psi = np.zeros(sp.dim, np.complex128)
        psi[si] = 1.0
        got = oapply.apply_targets(op, sp, psi, [ti])[0]
        want = _fermion_element(h1, h2, t, hf_bits, 2 * n_o)
        assert abs(got - want) < 1e-12
        if t == hf_bits:
            assert abs(got - e_hf) < 1e-12
