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


# ---------------------------------------------------------------- sparse route
# A few rotations on a basis state reach at most 2^k basis states, so at any
# qubit count the state, its energy and the gradient are exact sums over that
# support: E = sum_{s,t} conj(psi_t) psi_s <t|H|s> with
# <t|H|s> = sum_j c_j i^(#Y_j) (-1)^popcount(s & (Y|Z)_j) [t = s xor (X|Y)_j].

def sparse_state(rotations, theta, ref):
    """psi(theta) as {basis index: amplitude} (at most 64 qubits)."""
    from .apply import term_action

    flip, sign, n_y = term_action(np.asarray(rotations, dtype=np.uint8))
    psi = {int(ref): 1.0 + 0j}
    for k, th in enumerate(theta):
        nxt = {}
        for s, a in psi.items():
            nxt[s] = nxt.get(s, 0j) + np.cos(th) * a
            t = s ^ int(flip[k])
            sgn = -1.0 if bin(s & int(sign[k])).count("1") & 1 else 1.0
            nxt[t] = nxt.get(t, 0j) + 1j * np.sin(th) * a * (1j ** int(n_y[k] % 4)) * sgn
        psi = nxt
    return psi


def sparse_energy(op, rotations, theta, ref):
    from .apply import term_action

    psi = sparse_state(rotations, theta, ref)
    flip, sign, n_y = term_action(op.letters)
    factor = op.coeff * np.array([1, 1j, -1, -1j])[n_y % 4]
    e = 0j
    for s, a in psi.items():
        tgt = np.uint64(s) ^ flip
        par = np.bitwise_count(np.uint64(s) & sign) & 1
        contrib = factor * np.where(par == 1, -1.0, 1.0) * a
        for t, b in psi.items():
            hit = tgt == np.uint64(t)
            if hit.any():
                e += np.conj(b) * contrib[hit].sum()
    return float(e.real)


def sparse_gradient(op, rotations, theta, ref):
    """Parameter-shift gradient over the sparse energy."""
    theta = np.asarray(theta, dtype=np.float64)
    g = np.zeros_like(theta)
    for k in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += np.pi / 4
        tm[k] -= np.pi / 4
        g[k] = sparse_energy(op, rotations, tp, ref) - sparse_energy(op, rotations, tm, ref)
    return g
