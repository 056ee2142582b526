"""Pins of the oracle's short-iterative Lanczos propagation: agreement with a
dense matrix exponential, the free-fermion closed form at U = 0, norm and
energy conservation, and the exact result after a happy breakdown."""

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import apply as oapply
from oracle import jw as ojw
from oracle import krylov as okrylov
from oracle import space as ospace


def _hubbard(rows, cols, u):
    h1, h2 = synth.hubbard_spin_integrals(rows, cols, t=1.0, u=u, periodic=False)
    return ojw.jw_sum(h1, h2)


def _neel_state(rows, cols, sp):
    a, b = synth.neel_occupations(rows, cols)
    idx = sp.index_of(np.array([a | (b << (rows * cols))], np.uint64))[0]
    psi = np.zeros(sp.dim, np.complex128)
    psi[idx] = 1.0
    return psi


def _dense_sector(op, sp):
    basis_ops = np.eye(sp.dim, dtype=np.complex128)
    return np.stack([oapply.apply_scatter(op, sp, basis_ops[i]) for i in range(sp.dim)], axis=1)


@pytest.mark.parametrize("rows,cols,u", [(2, 2, 4.0), (2, 3, 4.0), (2, 3, 0.0)])
def test_krylov_matches_dense_expm(rows, cols, u):
    op = _hubbard(rows, cols, u)
    n = rows * cols
    na, nb = synth.neel_occupations(rows, cols)
    sp = ospace.SectorSpace(n, bin(na).count("1"), bin(nb).count("1"))
    Hd = _dense_sector(op, sp)
    np.testing.assert_allclose(Hd, Hd.conj().T, atol=1e-13)
    psi = synth.random_state(sp.dim, seed=7)
    dt = 0.05
    U = sla.expm(-1j * dt * Hd)
    out, e = okrylov.krylov_step(lambda v: oapply.apply_scatter(op, sp, v), psi, dt, m=12)
    np.testing.assert_allclose(out, U @ psi, atol=1e-12)
    assert abs(e - np.vdot(psi, Hd @ psi).real) < 1e-12


def test_free_fermion_occupations():
    """At U = 0 the Neel product state is a Slater determinant and the
    occupation of site i with spin sigma evolves as
    sum_{j occupied} |[exp(-i h t)]_ij|^2 with the hopping matrix h."""
    rows, cols = 2, 3
    n = rows * cols
    op = _hubbard(rows, cols, 0.0)
    na, nb = synth.neel_occupations(rows, cols)
    sp = ospace.SectorSpace(n, bin(na).count("1"), bin(nb).count("1"))
    psi = _neel_state(rows, cols, sp)
    h, _ = synth.hubbard_spatial_integrals(rows, cols, t=1.0, u=0.0, periodic=False)
    dt, steps = 0.05, 20
    for _ in range(steps):
        psi, _ = okrylov.krylov_step(lambda v: oapply.apply_scatter(op, sp, v), psi, dt, m=12)
    t = dt * steps
    prop = sla.expm(-1j * h * t)
    basis = sp.basis()
    prob = np.abs(psi) ** 2
    for sigma, occ_bits in ((0, na), (1, nb)):
        occ = [i for i in range(n) if (occ_bits >> i) & 1]
        want = (np.abs(prop[:, occ]) ** 2).sum(axis=1)
        got = np.array([prob[((basis >> np.uint64(i + sigma * n)) & np.uint64(1)) == 1].sum() for i in range(n)])
        np.testing.assert_allclose(got, want, atol=1e-11)


def test_conservation_and_breakdown():
    op = _hubbard(2, 3, 4.0)
    sp = ospace.SectorSpace(6, 2, 2)
    psi = synth.random_state(sp.dim, seed=9)
    app = lambda v: oapply.apply_scatter(op, sp, v)
    e0 = np.vdot(psi, app(psi)).real
    for _ in range(10):
        psi, _ = okrylov.krylov_step(app, psi, 0.05)
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-12
    assert abs(np.vdot(psi, app(psi)).real - e0) < 1e-11
    # an eigenvector: the Krylov space is one-dimensional and the step is exact
    Hd = _dense_sector(op, sp)
    w, U = np.linalg.eigh(Hd)
    v = U[:, 3].astype(np.complex128)
    V, alpha, beta, _ = okrylov.lanczos_basis(app, v, 12)
    assert len(alpha) == 1 and abs(alpha[0] - w[3]) < 1e-12
    out, _ = okrylov.krylov_step(app, v, 0.05)
    np.testing.assert_allclose(out, np.exp(-1j * w[3] * 0.05) * v, atol=1e-13)
