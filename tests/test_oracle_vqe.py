"""Pins of the oracle's Pauli-rotation ansatz: rotations against a library
matrix exponential, the parameter-shift gradient against central finite
differences, and the reference energy against the dense Hamiltonian."""

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import apply as oapply
from oracle import jw as ojw
from oracle import pauli as opauli
from oracle import vqe as ovqe


def _random_letters(rng, n, k):
    return [rng.integers(0, 4, n).astype(np.uint8) for _ in range(k)]


@pytest.mark.parametrize("n", [1, 3, 5])
def test_rotation_matches_matrix_exponential(n):
    rng = np.random.default_rng(n)
    for letters in _random_letters(rng, n, 6):
        P = opauli.dense_string(letters)
        theta = rng.normal()
        psi = synth.random_state(1 << n, seed=int(rng.integers(1 << 30)))
        want = sla.expm(1j * theta * P) @ psi
        got = ovqe.rotate(letters, theta, psi)
        np.testing.assert_allclose(got, want, atol=1e-12)


def test_rotation_inverse_and_quarter_turn():
    rng = np.random.default_rng(5)
    n = 4
    psi = synth.random_state(1 << n, seed=3)
    for letters in _random_letters(rng, n, 5):
        back = ovqe.rotate(letters, -0.37, ovqe.rotate(letters, 0.37, psi))
        np.testing.assert_allclose(back, psi, atol=1e-14)
        # exp(i pi/2 P) = i P
        np.testing.assert_allclose(ovqe.rotate(letters, np.pi / 2, psi), 1j * ovqe.pauli_apply(letters, psi),
                                   atol=1e-14)


def _small_problem(n_o=2, seed=3, n_rot=7):
    h1, h2 = synth.molecular_spin_integrals(n_o, seed=seed)
    op = ojw.jw_sum(h1, h2)
    n = 2 * n_o
    rng = np.random.default_rng(seed)
    rots = _random_letters(rng, n, n_rot)
    ref = 0b0101
    return op, rots, ref, rng.normal(size=n_rot) * 0.4


def test_parameter_shift_matches_finite_differences():
    op, rots, ref, theta = _small_problem()
    g = ovqe.gradient(op, rots, theta, ref)
    eps = 1e-6
    for k in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += eps
        tm[k] -= eps
        fd = (ovqe.energy(op, rots, tp, ref) - ovqe.energy(op, rots, tm, ref)) / (2 * eps)
        assert abs(fd - g[k]) < 1e-7 * max(1.0, abs(g[k]))


def test_reference_energy_is_diagonal_element():
    op, rots, ref, _ = _small_problem()
    H = oapply.dense_matrix(op)
    assert abs(ovqe.energy(op, rots, np.zeros(len(rots)), ref) - H[ref, ref].real) < 1e-12
    # a state built by rotations stays normalised and its energy is the dense quadratic form
    theta = np.linspace(-1, 1, len(rots))
    psi = ovqe.ansatz_state(rots, theta, ref, op.n_qubits)
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-13
    assert abs(ovqe.energy(op, rots, theta, ref) - np.vdot(psi, H @ psi).real) < 1e-12


def test_sparse_route_matches_dense_route():
    op, rots, ref, theta = _small_problem(n_o=3, seed=8, n_rot=4)
    dense = ovqe.ansatz_state(rots, theta, ref, op.n_qubits)
    sparse = ovqe.sparse_state(rots, theta, ref)
    assert len(sparse) <= 2 ** len(rots)
    emb = np.zeros_like(dense)
    for s, a in sparse.items():
        emb[s] += a
    np.testing.assert_allclose(emb, dense, atol=1e-14)
    assert abs(ovqe.sparse_energy(op, rots, theta, ref) - ovqe.energy(op, rots, theta, ref)) < 1e-12
    np.testing.assert_allclose(ovqe.sparse_gradient(op, rots, theta, ref), ovqe.gradient(op, rots, theta, ref),
                               atol=1e-12)
