"""GPU parity of the short-iterative Lanczos step (pbs_krylov_step) against
the oracle, plus the free-fermion closed form on the 4x4 Hubbard lattice at
U = 0 and conservation checks on the full 32-qubit sector."""

import numpy as np
import pytest
import scipy.linalg as sla
import torch

import synth
from oracle import apply as oapply
from oracle import jw as ojw
from oracle import krylov as okrylov
from oracle import space as ospace
from tests.conftest import rel_err

pytestmark = pytest.mark.gpu


def _api():
    from paper_2606_28952_amd import api

    return api


def _gpu_hubbard(dev, rows, cols, u, periodic):
    api = _api()
    h1, h2 = synth.hubbard_spin_integrals(rows, cols, t=1.0, u=u, periodic=periodic)
    return api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)).group(), (h1, h2)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("rows,cols,u,m", [(2, 3, 4.0, 12), (2, 2, 4.0, 12), (2, 3, 1.0, 5)])
def test_krylov_steps_match_oracle(dev, dtype, rows, cols, u, m):
    api = _api()
    G, (h1, h2) = _gpu_hubbard(dev, rows, cols, u, periodic=False)
    n = rows * cols
    na, nb = synth.neel_occupations(rows, cols)
    ka, kb = bin(na).count("1"), bin(nb).count("1")
    sp = api.Space.sector(n, ka, kb)
    osp = ospace.SectorSpace(n, ka, kb)
    op = ojw.jw_sum(h1, h2)
    psi = synth.random_state(osp.dim, seed=rows * 10 + cols)
    if dtype == torch.complex64:
        psi = psi.astype(np.complex64).astype(np.complex128)
    prop = api.KrylovPropagator(G, sp, dtype=dtype, m=m)
    t = torch.from_numpy(psi).to(dev).to(dtype)
    ref = psi.copy()
    for _ in range(5):
        info = prop.step(t, 0.05)
        ref, e = okrylov.krylov_step(lambda v: oapply.apply_scatter(op, osp, v), ref, 0.05, m=m)
        assert abs(info[1] - e) < (1e-12 if dtype == torch.complex128 else 1e-6) * max(1.0, abs(e))
    tol = 1e-11 if dtype == torch.complex128 else 2e-6
    assert rel_err(t.cpu().numpy(), ref) < tol


def test_krylov_breakdown_on_eigenvector(dev):
    api = _api()
    G, (h1, h2) = _gpu_hubbard(dev, 2, 3, 4.0, periodic=False)
    osp = ospace.SectorSpace(6, 2, 2)
    op = ojw.jw_sum(h1, h2)
    eye = np.eye(osp.dim, dtype=np.complex128)
    Hd = np.stack([oapply.apply_scatter(op, osp, eye[i]) for i in range(osp.dim)], axis=1)
    w, U = np.linalg.eigh(Hd)
    v = U[:, 0].astype(np.complex128)
    sp = api.Space.sector(6, 2, 2)
    prop = api.KrylovPropagator(G, sp, dtype=torch.complex128, m=12)
    t = torch.from_numpy(v).to(dev)
    info = prop.step(t, 0.05)
    assert info[2] == 1.0
    assert rel_err(t.cpu().numpy(), np.exp(-1j * w[0] * 0.05) * v) < 1e-12


def test_krylov_rejects_bad_arguments(dev):
    api = _api()
    from paper_2606_28952_amd._abi import PbsError

    G, _ = _gpu_hubbard(dev, 2, 2, 4.0, periodic=False)
    sp = api.Space.sector(4, 2, 2)
    with pytest.raises(PbsError, match="m must be"):
        api.KrylovPropagator(G, sp, m=17)
    prop = api.KrylovPropagator(G, sp, dtype=torch.complex64, m=4)
    with pytest.raises(TypeError):
        prop.step(torch.zeros(sp.dim, dtype=torch.complex128, device=dev), 0.05)


def _site_occupations(space, psi, n_sites):
    """<n_{i,sigma}> for all sites and both spins from the sector state."""
    api = _api()
    dim = psi.numel()
    prob = (psi.real.to(torch.float64) ** 2 + psi.imag.to(torch.float64) ** 2)
    occ = np.zeros((2, n_sites))
    chunk = 1 << 24
    for start in range(0, dim, chunk):
        idx = torch.arange(start, min(dim, start + chunk), dtype=torch.int64, device=psi.device)
        bits = space.unrank(idx)
        p = prob[start:start + idx.numel()]
        for sigma in range(2):
            for i in range(n_sites):
                sel = ((bits >> (i + sigma * n_sites)) & 1).to(torch.float64)
                occ[sigma, i] += float(torch.dot(sel, p))
    return occ


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-10), (torch.complex64, 2e-5)])
def test_hubbard_4x4_free_fermions(dev, dtype, tol):
    """4x4 periodic lattice at U = 0, (8, 8) sector (D = 165,636,900): from the
    Neel product state, site occupations follow sum_{j occupied}
    |[exp(-i h t)]_ij|^2 for the 16x16 hopping matrix h."""
    api = _api()
    rows = cols = 4
    n = 16
    G, _ = _gpu_hubbard(dev, rows, cols, 0.0, periodic=True)
    sp = api.Space.sector(n, 8, 8)
    na, nb = synth.neel_occupations(rows, cols)
    start = sp.rank(torch.tensor([na | (nb << n)], dtype=torch.int64, device=dev)).item()
    psi = torch.zeros(sp.dim, dtype=dtype, device=dev)
    psi[start] = 1.0
    prop = api.KrylovPropagator(G, sp, dtype=dtype, m=12)
    dt, steps = 0.05, 6
    energies = []
    for _ in range(steps):
        info = prop.step(psi, dt)
        energies.append(info[1])
    torch.cuda.synchronize()
    nrm = float(torch.linalg.vector_norm(psi.to(torch.complex128)).item())
    assert abs(nrm - 1.0) < tol
    assert max(energies) - min(energies) < 10 * tol
    h, _ = synth.hubbard_spatial_integrals(rows, cols, t=1.0, u=0.0, periodic=True)
    prop_h = sla.expm(-1j * h * dt * steps)
    got = _site_occupations(sp, psi, n)
    for sigma, bits in ((0, na), (1, nb)):
        occ = [i for i in range(n) if (bits >> i) & 1]
        want = (np.abs(prop_h[:, occ]) ** 2).sum(axis=1)
        np.testing.assert_allclose(got[sigma], want, atol=tol)
