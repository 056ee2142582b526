"""Jordan-Wigner Hamiltonian by the conventional route (oracle; test use only).

Section 2.3 gives the mapping a+_p = 1/2 (X_p - i Y_p) Z_{p-1} ... Z_0 and
a_p = 1/2 (X_p + i Y_p) Z_{p-1} ... Z_0.  The paper builds the qubit
Hamiltonian with precomputed 4/16-string expansions (Algorithm 1); this oracle
instead follows the "conventional implementation" the same section describes:
every ladder operator is a two-term Pauli sum, the sums of each integral's
fermionic product are multiplied letter by letter, all contributions are
collected and the whole list is reduced once to canonical form.

The Hamiltonian is Eq. second_quantized_hamiltonian written over spin-orbitals,
    H = e0 I + sum_PQ h1[P,Q] a+_P a_Q + 1/2 sum_PQRS h2[P,Q,R,S] a+_P a+_Q a_R a_S,
with an integral kept when |h| > eps (Algorithm 1's threshold test, read as a
strict inequality; eps = 0 keeps every nonzero integral).  e0 is the
identity coefficient (E_NN of the same equation).  Every contribution is an
integral times a power of two times a power of i, hence exact in float64, so
the correctly rounded canonical sums do not depend on the order of the loops.
"""

import numpy as np

from .pauli import I, X, Y, Z, PauliSum, canonical_arrays, string_product, I_POW


def ladder(n, p, dagger):
    """a+_p (dagger=True) or a_p as letter rows [2, n] and magnitudes/phases.

    Term 0: X_p Z_{<p} with coefficient 1/2; term 1: Y_p Z_{<p} with
    coefficient -i/2 for a+_p and +i/2 for a_p.  Returned as
    (letters [2, n], phase exponents [2]) with common magnitude 1/2."""
    rows = np.zeros((2, n), dtype=np.uint8)
    rows[:, :p] = Z
    rows[0, p] = X
    rows[1, p] = Y
    phase = np.array([0, 3 if dagger else 1], dtype=np.uint8)
    return rows, phase


def ladder_sum(n, p, dagger):
    rows, phase = ladder(n, p, dagger)
    return PauliSum(n, rows, 0.5 * I_POW[phase])


def _products(n, factors, scale):
    """Expand prod_f (1/2)(term0_f + term1_f) for a batch of index tuples.

    factors: list of (indices [K], dagger) applied left to right; scale: float64
    [K] (the integral including the 1/2 of the two-body sum).  Returns letter
    rows [K * 2^F, n] and exact complex coefficients."""
    ladders = {True: [ladder(n, p, True) for p in range(n)],
               False: [ladder(n, p, False) for p in range(n)]}
    k = len(scale)
    f = len(factors)
    rows_all = []
    coeff_all = []
    for combo in range(1 << f):
        letters = np.zeros((k, n), dtype=np.uint8)
        phase = np.zeros(k, dtype=np.uint8)
        for pos, (idx, dagger) in enumerate(factors):
            which = (combo >> pos) & 1
            lrows = np.stack([ladders[dagger][int(p)][0][which] for p in range(n)])
            lphase = np.array([ladders[dagger][int(p)][1][which] for p in range(n)], dtype=np.uint8)
            letters, phase = string_product(letters, phase, lrows[idx], lphase[idx])
        mag = scale * (0.5 ** f)            # exact: power-of-two scaling
        re = np.where(phase == 0, mag, np.where(phase == 2, -mag, 0.0))
        im = np.where(phase == 1, mag, np.where(phase == 3, -mag, 0.0))
        rows_all.append(letters)
        coeff_all.append(re + 1j * im)
    return np.concatenate(rows_all), np.concatenate(coeff_all)


def jw_contributions(h1, h2, e0=0.0, eps=0.0):
    """All unreduced (letters, coeff) contributions of the JW Hamiltonian."""
    h1 = np.asarray(h1, dtype=np.float64)
    h2 = np.asarray(h2, dtype=np.float64)
    n = h1.shape[0]
    rows = [np.zeros((1, n), dtype=np.uint8)]
    coeffs = [np.array([complex(e0)])]
    p, q = np.nonzero(np.abs(h1) > eps)
    if len(p):
        r1, c1 = _products(n, [(p, True), (q, False)], h1[p, q])
        rows.append(r1)
        coeffs.append(c1)
    P, Q, R, S = np.nonzero(np.abs(h2) > eps)
    if len(P):
        r2, c2 = _products(n, [(P, True), (Q, True), (R, False), (S, False)], 0.5 * h2[P, Q, R, S])
        rows.append(r2)
        coeffs.append(c2)
    return PauliSum(n, np.concatenate(rows), np.concatenate(coeffs))


def jw_hamiltonian(h1, h2, e0=0.0, eps=0.0, eps_drop=0.0):
    """Canonical (x [M,W], z [M,W], coeff [M]) of the JW qubit Hamiltonian."""
    return canonical_arrays(jw_contributions(h1, h2, e0, eps), eps_drop)


def jw_sum(h1, h2, e0=0.0, eps=0.0, eps_drop=0.0):
    """Same as jw_hamiltonian, returned as a letter-form PauliSum."""
    from .pauli import canonicalize
    return canonicalize(jw_contributions(h1, h2, e0, eps), eps_drop)
