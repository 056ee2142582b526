"""Pins of the oracle's C twin (oracle/capply.c): dense Kronecker brute force
for n <= 10, equality with the NumPy oracle on the 12-qubit molecular
workload (full space and sector) and on 16- and 20-qubit sectors, target
gather = source scatter, scatter from a support list = scatter of the whole
vector, thread-count independence, and the sector as a restriction of the
full space for a number-conserving operator."""

import numpy as np
import pytest

import synth
from oracle import apply as oapply
from oracle import jw, native, space
from oracle.pauli import PauliSum


def _random_sum(n, m, seed):
    letters, _ = synth.random_pauli_strings(m, n, seed)
    rng = np.random.default_rng(seed + 1)
    c = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    return PauliSum(n, letters, c.astype(np.complex128))


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("n,m", [(1, 3), (2, 7), (5, 30), (8, 60), (10, 40)])
def test_dense_brute_force(n, m):
    op = _random_sum(n, m, seed=500 + n)
    psi = synth.random_state(1 << n, seed=600 + n)
    want = op.dense() @ psi
    full = space.FullSpace(n)
    got, _ = native.apply_scatter(op, full, psi, threads=3)
    assert _rel(got, want) < 1e-13
    tg, _ = native.apply_targets(op, full, psi, np.arange(1 << n), threads=2)
    assert _rel(tg, want) < 1e-13


def test_twelve_qubit_molecular_equals_numpy_oracle():
    h1, h2 = synth.molecular_spin_integrals(6, seed=1001)
    op = jw.jw_sum(h1, h2)
    for sp, seed in [(space.FullSpace(12), 1101), (space.SectorSpace(6, 3, 3), 1102)]:
        psi = synth.random_state(sp.dim, seed)
        ref = oapply.apply_scatter(op, sp, psi)
        got, _ = native.apply_scatter(op, sp, psi)
        assert _rel(got, ref) < 1e-13
        tg, _ = native.apply_targets(op, sp, psi, np.arange(sp.dim))
        assert _rel(tg, ref) < 1e-13


@pytest.mark.parametrize("n_o,na,nb", [(8, 4, 4), (10, 5, 5)])
def test_sector_equals_numpy_oracle(n_o, na, nb):
    """16 and 20 qubits: the whole sector vector against the NumPy scatter
    (for 20 qubits on the first 2,000 canonical strings, to keep the NumPy
    side within seconds)."""
    h1, h2 = synth.molecular_spin_integrals(n_o, seed=40 + n_o)
    op = jw.jw_sum(h1, h2)
    if n_o == 10:
        op = PauliSum(op.n_qubits, op.letters[:2000], op.coeff[:2000])
    sp = space.SectorSpace(n_o, na, nb)
    psi = synth.random_state(sp.dim, seed=7 + n_o)
    ref = oapply.apply_scatter(op, sp, psi)
    got, used = native.apply_scatter(op, sp, psi, threads=4)
    assert used == 4
    assert _rel(got, ref) < 1e-13
    rows = np.random.default_rng(n_o).choice(sp.dim_alpha, 3, replace=False)
    tgt = (rows[:, None] * sp.dim_beta + np.arange(sp.dim_beta)[None, :]).reshape(-1)
    tg, _ = native.apply_targets(op, sp, psi, tgt, threads=4)
    assert _rel(tg, ref[tgt]) < 1e-13


def test_sparse_support_and_thread_counts():
    """Scatter from a support list equals the scatter of the vector that is
    zero elsewhere; the thread count only reorders the final sums."""
    h1, h2 = synth.molecular_spin_integrals(7, seed=77)
    op = jw.jw_sum(h1, h2)
    sp = space.SectorSpace(7, 3, 4)
    rng = np.random.default_rng(5)
    support = np.sort(rng.choice(sp.dim, 200, replace=False))
    psi = np.zeros(sp.dim, np.complex128)
    psi[support] = rng.standard_normal(200) + 1j * rng.standard_normal(200)
    whole, _ = native.apply_scatter(op, sp, psi, threads=1)
    part, _ = native.apply_scatter(op, sp, psi, sources=support, threads=5)
    assert _rel(part, whole) < 1e-14
    assert _rel(whole, oapply.apply_scatter(op, sp, psi)) < 1e-13


def test_sector_is_restriction_of_full_space():
    h1, h2 = synth.molecular_spin_integrals(5, seed=55)
    op = jw.jw_sum(h1, h2)
    sec = space.SectorSpace(5, 2, 3)
    psi = synth.random_state(sec.dim, 8)
    full_out, _ = native.apply_scatter(op, space.FullSpace(10), oapply.embed(psi, sec, 10))
    got, _ = native.apply_scatter(op, sec, psi)
    assert _rel(got, oapply.restrict(full_out, sec)) < 1e-14
    # nothing leaks out of the sector for a number- and S_z-conserving H
    outside = np.delete(full_out, sec.basis().astype(np.int64))
    assert np.abs(outside).max() < 1e-14
