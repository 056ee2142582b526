"""Pins of the oracle's Pauli algebra against facts fixed outside the oracle:
the single-qubit table, dense Kronecker matrices, commutation, associativity
and exact summation."""

import math

import numpy as np
import pytest

import synth
from oracle import pauli
from oracle.pauli import PauliSum
from tests.conftest import golden_rows

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")

SIGMA = {
    "I": np.eye(2, dtype=complex),
    "X": np.array([[0, 1], [1, 0]], dtype=complex),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=complex),
    "Z": np.array([[1, 0], [0, -1]], dtype=complex),
}


def test_single_qubit_mapping_golden():
    for a, b, letter, tx, ty, tz in golden_rows("single_qubit_mapping.txt"):
        row = pauli.parse(letter)
        x, z = pauli.letters_to_xz(row[None, :])
        assert (int(x[0, 0]), int(z[0, 0])) == (int(a), int(b))
        # type recovery equations of Section 2.2
        ia, ib = int(a), int(b)
        t_y = ia & ib
        assert (ia ^ t_y, t_y, ib ^ t_y) == (int(tx), int(ty), int(tz))
        assert pauli.to_text(pauli.xz_to_letters(x, z, 1)[0]) == letter


def test_single_qubit_products_golden():
    for left, right, result, phase in golden_rows("single_qubit_products.txt"):
        letters, ph = pauli.string_product(pauli.parse(left), 0, pauli.parse(right), 0)
        assert pauli.to_text(letters) == result
        assert int(ph) == int(phase)
        # and the matrices agree
        lhs = SIGMA[left] @ SIGMA[right]
        rhs = (1j ** int(phase)) * SIGMA[result]
        np.testing.assert_array_equal(lhs, rhs)


def test_square_is_identity():
    letters, _ = synth.random_pauli_strings(50, 9, seed=1)
    sq, ph = pauli.string_product(letters, 0, letters, 0)
    assert (sq == 0).all() and (ph == 0).all()


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6])
def test_product_matches_dense(n):
    la, pa = synth.random_pauli_strings(40, n, seed=10 + n)
    lb, pb = synth.random_pauli_strings(40, n, seed=20 + n)
    lc, pc = pauli.string_product(la, pa, lb, pb)
    for k in range(40):
        lhs = pauli.dense_string(la[k], pa[k]) @ pauli.dense_string(lb[k], pb[k])
        rhs = pauli.dense_string(lc[k], pc[k])
        np.testing.assert_array_equal(lhs, rhs)


def test_dense_qubit_order():
    # qubit 0 is bit 0 of the basis index: X on qubit 0 maps |0> to |1>
    m = pauli.dense_string(pauli.parse("XI"))
    assert m[1, 0] == 1 and m[2, 0] == 0
    m = pauli.dense_string(pauli.parse("IX"))
    assert m[2, 0] == 1


def _symplectic_form(la, lb):
    xa, za = pauli.letters_to_xz(la[None, :])
    xb, zb = pauli.letters_to_xz(lb[None, :])
    w = 0
    for i in range(xa.shape[1]):
        w += bin(int(xa[0, i]) & int(zb[0, i])).count("1") + bin(int(za[0, i]) & int(xb[0, i])).count("1")
    return w % 2


@pytest.mark.parametrize("n", [2, 4, 6])
def test_commutation_symplectic(n):
    la, _ = synth.random_pauli_strings(60, n, seed=30 + n)
    lb, _ = synth.random_pauli_strings(60, n, seed=40 + n)
    for k in range(60):
        A, B = pauli.dense_string(la[k]), pauli.dense_string(lb[k])
        omega = _symplectic_form(la[k], lb[k])
        np.testing.assert_array_equal(A @ B, (-1) ** omega * (B @ A))
        assert pauli.commutes(la[k], lb[k]) == (omega == 0)


def test_associativity_multiword():
    n = 130
    la, pa = synth.random_pauli_strings(30, n, seed=50)
    lb, pb = synth.random_pauli_strings(30, n, seed=51)
    lc, pc = synth.random_pauli_strings(30, n, seed=52)
    l1, p1 = pauli.string_product(*pauli.string_product(la, pa, lb, pb), lc, pc)
    l2, p2 = pauli.string_product(la, pa, *pauli.string_product(lb, pb, lc, pc))
    np.testing.assert_array_equal(l1, l2)
    np.testing.assert_array_equal(p1, p2)


def test_multiword_product_factorises_per_qubit():
    # a 130-qubit product equals the per-qubit products, phases added
    n = 130
    la, _ = synth.random_pauli_strings(10, n, seed=53)
    lb, _ = synth.random_pauli_strings(10, n, seed=54)
    lc, pc = pauli.string_product(la, 0, lb, 0)
    for k in range(10):
        total = 0
        for q in range(n):
            l1, p1 = pauli.string_product(la[k, q:q + 1], 0, lb[k, q:q + 1], 0)
            assert l1[0] == lc[k, q]
            total += int(p1)
        assert total % 4 == int(pc[k])


def test_xz_roundtrip_multiword():
    letters, _ = synth.random_pauli_strings(25, 130, seed=55)
    x, z = pauli.letters_to_xz(letters)
    assert x.shape == (25, 3)
    np.testing.assert_array_equal(pauli.xz_to_letters(x, z, 130), letters)
    # bit k of word w is qubit 64 w + k
    row = np.zeros(130, np.uint8)
    row[70] = pauli.X
    row[129] = pauli.Z
    x1, z1 = pauli.letters_to_xz(row[None])
    assert int(x1[0, 1]) == 1 << 6 and int(z1[0, 2]) == 1 << 1


def test_canonicalize_exact_sum_and_order():
    terms = [("XZ", 1e100), ("ZI", 2.0), ("XZ", 1.0), ("XZ", -1e100), ("IY", 0.0), ("ZI", -2.0)]
    s = PauliSum.from_text(terms)
    c = pauli.canonicalize(s)
    d = c.as_dict()
    assert d == {"XZ": 1.0 + 0j}
    # exact zero kept only with a negative threshold
    c2 = pauli.canonicalize(s, eps_drop=-1.0)
    assert set(c2.as_dict()) == {"XZ", "ZI", "IY"}
    assert math.copysign(1.0, c2.as_dict()["ZI"].real) == 1.0  # +0.0


def test_canonicalize_sorted_by_x_then_z():
    letters, _ = synth.random_pauli_strings(300, 7, seed=60)
    coeff = np.random.default_rng(61).standard_normal(300) + 0j
    x, z, c = pauli.canonical_arrays(PauliSum(7, letters, coeff))
    keys = [(int(a), int(b)) for a, b in zip(x[:, 0], z[:, 0])]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)


def test_canonicalize_permutation_invariant_and_idempotent():
    rng = np.random.default_rng(62)
    letters, _ = synth.random_pauli_strings(500, 5, seed=63)
    coeff = rng.standard_normal(500) * 10.0 ** rng.integers(-8, 8, 500) + 1j * rng.standard_normal(500)
    s = PauliSum(5, letters, coeff)
    x1, z1, c1 = pauli.canonical_arrays(s)
    perm = rng.permutation(500)
    x2, z2, c2 = pauli.canonical_arrays(PauliSum(5, letters[perm], coeff[perm]))
    np.testing.assert_array_equal(x1, x2)
    np.testing.assert_array_equal(z1, z2)
    assert c1.tobytes() == c2.tobytes()
    again = pauli.canonicalize(pauli.canonicalize(s))
    assert again.coeff.tobytes() == c1.tobytes()


def test_drop_threshold_max_norm():
    s = PauliSum.from_text([("X", 1e-3 + 1e-9j), ("Z", 1e-9 + 1e-9j), ("Y", 1e-9 - 1e-2j)])
    d = pauli.canonicalize(s, eps_drop=1e-6).as_dict()
    assert set(d) == {"X", "Y"}


@pytest.mark.parametrize("n", [3, 4])
def test_sum_product_matches_dense(n):
    rng = np.random.default_rng(70 + n)
    la, _ = synth.random_pauli_strings(12, n, seed=71 + n)
    lb, _ = synth.random_pauli_strings(9, n, seed=72 + n)
    A = PauliSum(n, la, rng.standard_normal(12) + 1j * rng.standard_normal(12))
    B = PauliSum(n, lb, rng.standard_normal(9) + 1j * rng.standard_normal(9))
    x, z, c = pauli.sum_product_canonical(A, B)
    C = PauliSum(n, pauli.xz_to_letters(x, z, n), c)
    np.testing.assert_allclose(C.dense(), A.dense() @ B.dense(), atol=1e-13)
    # unreduced product has the same dense matrix
    np.testing.assert_allclose(pauli.sum_product(A, B).dense(), A.dense() @ B.dense(), atol=1e-13)


def test_sum_product_correct_rounding():
    # cancellation that float products would lose: exact rational result rounded once
    e = 2.0 ** -30
    A = PauliSum.from_text([("X", 1.0 + e), ("Y", 1.0)])
    B = PauliSum.from_text([("X", 1.0 - e), ("Y", -1.0)])
    # XX = I, YY = I, XY = iZ, YX = -iZ
    x, z, c = pauli.sum_product_canonical(A, B)
    d = {(int(a[0]), int(b[0])): v for a, b, v in zip(x, z, c)}
    # I coefficient: (1+e)(1-e) - 1 = -e^2 exactly; a rounded product would give 0
    assert (1.0 + e) * (1.0 - e) - 1.0 == 0.0
    assert d[(0, 0)] == complex(-(e * e), 0.0)
    # Z coefficient: i[-(1+e) - (1-e)] = -2i
    assert d[(0, 1)] == complex(0.0, -2.0)


def _xz_dense(n, xg, offsets, z, c):
    """Dense matrix of sum_k C_k X^x_k Z^z_k from the bit action of the XZ form,
    X^x Z^z |s> = (-1)^popcount(z & s) |s xor x>, written without letters."""
    dim = 1 << n
    s = np.arange(dim, dtype=np.uint64)
    out = np.zeros((dim, dim), dtype=np.complex128)
    for g in range(len(xg)):
        tgt = (s ^ np.uint64(xg[g])).astype(np.int64)
        for k in range(int(offsets[g]), int(offsets[g + 1])):
            sign = 1.0 - 2.0 * (np.bitwise_count(s & np.uint64(z[k])) & 1)
            out[tgt, s.astype(np.int64)] += c[k] * sign
    return out


@pytest.mark.parametrize("n,m,seed", [(1, 4, 1), (3, 20, 2), (5, 60, 3), (6, 120, 4)])
def test_group_by_x_xz_coefficients_match_dense(n, m, seed):
    """Section 2.3 (C_j = c_j Lambda_j) and Eq. topological_group: the grouped
    XZ-form coefficients rebuild the operator; conjugating Lambda (i^-#Y
    instead of i^+#Y) or dropping it fails for every string containing Y."""
    letters, _ = synth.random_pauli_strings(m, n, seed)
    rng = np.random.default_rng(seed)
    op = PauliSum(n, letters, rng.standard_normal(m) + 1j * rng.standard_normal(m))
    x, z, c = pauli.canonical_arrays(op)
    xg, offsets, zk, ck = pauli.group_by_x(x, z, c)
    assert np.all(np.diff(xg.astype(np.int64)) > 0)          # one group per X, ascending
    assert int(offsets[-1]) == len(c)
    np.testing.assert_allclose(_xz_dense(n, xg, offsets, zk, ck), op.dense(), rtol=0, atol=1e-13)


def test_group_by_x_jw_operator_matches_dense():
    from oracle import jw

    h1, h2 = synth.molecular_spin_integrals(3, seed=31)
    x, z, c = jw.jw_hamiltonian(h1, h2)
    xg, offsets, zk, ck = pauli.group_by_x(x, z, c)
    op = jw.jw_sum(h1, h2)
    np.testing.assert_allclose(_xz_dense(6, xg, offsets, zk, ck), op.dense(), rtol=0, atol=1e-12)
    # a real Hermitian JW operator has an even number of Y per string; strings
    # with two Y (Lambda = -1) are there, so dropping Lambda fails this test
    # (odd counts, where conjugating Lambda shows, are covered by the random sums)
    assert np.any(np.bitwise_count(x[:, 0] & z[:, 0]) % 4 == 2)
