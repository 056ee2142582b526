"""Pauli-rotation ansatz, its energy and gradient (oracle; test use only).

The ansatz is psi(theta) = R_{n-1} ... R_0 |ref> with
R_k = exp(i theta_k P_k) = cos(theta_k) I + i sin(theta_k) P_k for Hermitian
Pauli strings P_k (P_k^2 = I), and the energy is E = <psi|H|psi> (Section
2.1, Eq. vqe_energy).  Each P_k acts through the letter-by-letter rule of
``oracle.apply`` on the full 2^n space; H|psi> is the term-by-term scatter of
``oracle.apply.apply_scatter``.  Because every rotation generator squares to
the identity, E is a + b cos(2 theta_k) + c sin(2 theta_k) in each parameter,
so the exact gradient is the parameter-shift difference
dE/dtheta_k = E(theta + pi/4 e_k) - E(theta - pi/4 e_k).  All arithmetic is
float64.
"""

import numpy as np

from .apply import apply_scatter
from .pauli import PauliSum
from .space import FullSpace


def pauli_apply(letters, psi):
    """P psi for one letter-form string (coefficient 1) on the full space."""
    letters = np.asarray(letters, dtype=np.uint8).reshape(1, -1)
    n = letters.shape[1]
    return apply_scatter(PauliSum(n, letters, np.array([1.0 + 0j])), FullSpace(n), psi)


def rotate(letters, theta, psi):
    """exp(i theta P) psi = cos(theta) psi + i sin(theta) P psi."""
    return np.cos(theta) * psi + 1j * np.sin(theta) * pauli_apply(letters, psi)


def ansatz_state(rotations, theta, ref, n_qubits):
    psi = np.zeros(1 << n_qubits, dtype=np.complex128)
    psi[ref] = 1.0
    for letters, th in zip(rotations, theta):
        psi = rotate(letters, th, psi)
    return psi


def energy(op, rotations, theta, ref):
    psi = ansatz_state(rotations, theta, ref, op.n_qubits)
    return float(np.vdot(psi, apply_scatter(op, FullSpace(op.n_qubits), psi)).real)


def gradient(op, rotations, theta, ref):
    """Exact gradient by the parameter-shift rule (two energies per parameter)."""
    theta = np.asarray(theta, dtype=np.float64)
    g = np.zeros_like(theta)
    for k in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += np.pi / 4
        tm[k] -= np.pi / 4
        g[k] = energy(op, rotations, tp, ref) - energy(op, rotations, tm, ref)
    return g
