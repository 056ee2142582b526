"""Pins of the oracle's operator application: dense Kronecker brute force,
the sector as a restriction of the full space, target-gather equals
source-scatter, Hermiticity, P^2 = I and closed-form TFIM energies."""

import numpy as np
import pytest
import scipy.sparse as sps

import synth
from oracle import apply as oapply
from oracle import jw, pauli, space
from oracle.pauli import PauliSum


def _random_sum(n, m, seed, hermitian=False):
    letters, _ = synth.random_pauli_strings(m, n, seed)
    rng = np.random.default_rng(seed + 1)
    c = rng.standard_normal(m) + (0 if hermitian else 1j * rng.standard_normal(m))
    return PauliSum(n, letters, c.astype(np.complex128))


@pytest.mark.parametrize("n,m", [(1, 3), (3, 10), (6, 40), (8, 60), (10, 30)])
def test_full_space_dense(n, m):
    op = _random_sum(n, m, seed=200 + n)
    psi = synth.random_state(1 << n, seed=300 + n)
    got = oapply.apply_scatter(op, space.FullSpace(n), psi)
    want = op.dense() @ psi
    assert np.linalg.norm(got - want) <= 1e-13 * max(1.0, np.linalg.norm(want))


def _sparse_kron(op):
    mats = {0: sps.identity(2, format="csr", dtype=complex),
            1: sps.csr_matrix(np.array([[0, 1], [1, 0]], dtype=complex)),
            2: sps.csr_matrix(np.array([[0, -1j], [1j, 0]], dtype=complex)),
            3: sps.csr_matrix(np.array([[1, 0], [0, -1]], dtype=complex))}
    n = op.n_qubits
    total = None
    for row, c in zip(op.letters, op.coeff):
        m = sps.identity(1, format="csr", dtype=complex)
        for letter in row[::-1]:
            m = sps.kron(m, mats[int(letter)], format="csr")
        total = c * m if total is None else total + c * m
    return total


def test_twelve_qubit_molecular_sparse_kron():
    h1, h2 = synth.molecular_spin_integrals(6, seed=1001)
    op = jw.jw_sum(h1, h2)
    assert op.n_terms == 1819
    Hs = _sparse_kron(op)
    full = space.FullSpace(12)
    psi = synth.random_state(4096, seed=1101)
    got = oapply.apply_scatter(op, full, psi)
    want = Hs @ psi
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
    # sector (3, 3): restriction of the full-space result (H conserves N_alpha, N_beta)
    sec = space.SectorSpace(6, 3, 3)
    phi = synth.random_state(400, seed=1102)
    got_s = oapply.apply_scatter(op, sec, phi)
    want_full = Hs @ oapply.embed(phi, sec, 12)
    assert np.linalg.norm(got_s - oapply.restrict(want_full, sec)) <= 1e-12 * np.linalg.norm(want_full)
    # nothing leaks outside the sector
    outside = np.ones(4096, bool)
    outside[sec.basis().astype(np.int64)] = False
    assert np.abs(want_full[outside]).max() < 1e-12


def test_sector_is_projection_for_nonconserving_operator():
    n_o = 3
    op = _random_sum(2 * n_o, 25, seed=400)
    sec = space.SectorSpace(n_o, 1, 2)
    phi = synth.random_state(sec.dim, seed=401)
    got = oapply.apply_scatter(op, sec, phi)
    want = oapply.restrict(op.dense() @ oapply.embed(phi, sec, 2 * n_o), sec)
    np.testing.assert_allclose(got, want, atol=1e-13)


@pytest.mark.parametrize("kind", ["full", "sector"])
def test_target_gather_equals_source_scatter(kind):
    if kind == "full":
        op = _random_sum(9, 80, seed=500)
        sp = space.FullSpace(9)
    else:
        h1, h2 = synth.molecular_spin_integrals(5, seed=501)
        op = jw.jw_sum(h1, h2)
        sp = space.SectorSpace(5, 2, 3)
    psi = synth.random_state(sp.dim, seed=502)
    full = oapply.apply_scatter(op, sp, psi)
    idx = np.random.default_rng(503).choice(sp.dim, size=min(60, sp.dim), replace=False)
    np.testing.assert_allclose(oapply.apply_targets(op, sp, psi, idx), full[idx], atol=1e-13)


def test_hermiticity_and_expval():
    h1, h2 = synth.molecular_spin_integrals(4, seed=600)
    op = jw.jw_sum(h1, h2)
    sp = space.SectorSpace(4, 2, 2)
    a = synth.random_state(sp.dim, 601)
    b = synth.random_state(sp.dim, 602)
    lhs = np.vdot(b, oapply.apply_scatter(op, sp, a))
    rhs = np.conj(np.vdot(a, oapply.apply_scatter(op, sp, b)))
    assert abs(lhs - rhs) < 1e-13
    e, nrm = oapply.expval(op, sp, a)
    assert abs(e.imag) < 1e-13 and abs(nrm - 1) < 1e-14
    # E(e_s) is the diagonal element
    basis = np.zeros(sp.dim, np.complex128)
    basis[7] = 1.0
    e7, _ = oapply.expval(op, sp, basis)
    assert abs(e7 - oapply.apply_targets(op, sp, basis, [7])[0]) < 1e-14


def test_single_string_squares_to_identity():
    letters, phase = synth.random_pauli_strings(20, 8, seed=700)
    psi = synth.random_state(256, 701)
    sp = space.FullSpace(8)
    for row in letters:
        op = PauliSum(8, row[None, :], np.array([1.0 + 0j]))
        twice = oapply.apply_scatter(op, sp, oapply.apply_scatter(op, sp, psi))
        np.testing.assert_allclose(twice, psi, atol=1e-15)


def test_tfim_closed_forms():
    n = 12
    terms = synth.tfim_terms(n)
    op = PauliSum.from_text(terms)
    x, z, c = pauli.canonical_arrays(op)
    assert len(c) == 2 * n - 1 and len(np.unique(x[:, 0])) == n + 1
    sp = space.FullSpace(n)
    zero = np.zeros(1 << n, np.complex128)
    zero[0] = 1.0
    e0, _ = oapply.expval(op, sp, zero)
    assert abs(e0 - 0.25 * (n - 1)) < 1e-13              # all spins up: J (N-1)
    plus = np.full(1 << n, 2.0 ** (-n / 2), np.complex128)
    ep, _ = oapply.expval(op, sp, plus)
    assert abs(ep - 1.0 * n) < 1e-12                     # |+...+>: h N
