"""Full-size parity of the sector apply and the fused energy, through the C
ABI, against the oracle's C twin (oracle/capply.c), in the launch
configuration the benchmark times.

* 28-qubit molecular sector (n_orb = 14, (7, 7), D = 11,778,624, 55,371
  strings): every target of 64 whole alpha rows (the first, the last and 62
  seeded ones; each row spans all seven 512-column chunks including the
  360-column tail) for a dense random state, and the WHOLE output vector
  plus the energy for a state supported on 8 whole rows and 500 scattered
  configurations (the oracle scatters from the support, which gives every
  output amplitude exactly).
* 32-qubit 4x4 Hubbard sector ((8, 8), D = 165,636,900): 16 whole rows of
  12,870 columns for a dense state, and the whole vector for a state
  supported on 4 rows.
* One device's share of an eight-way split of the target alpha rows at both
  sizes (the row-range entry points), bit-identical to those rows of the
  whole-sector apply.

Bars: complex128 storage within 1e-12 of the oracle in the relative 2-norm;
complex64 storage within 1e-6 of the oracle run on the same FP32-rounded
input (only each output's final rounding to FP32 remains); energies from the
fused float64 reduction within 1e-12 relative (complex128) and 1e-8 Ha
absolute (complex64) of the oracle's vdot(psi, H psi) on identical inputs."""

import numpy as np
import pytest
import torch

import synth
from oracle import jw as ojw
from oracle import native
from oracle import space as ospace
from tests.conftest import rel_err

pytestmark = pytest.mark.gpu


def _api():
    from paper_2606_28952_amd import api

    return api


def _row_targets(rows, dim_beta):
    rows = np.asarray(rows, dtype=np.int64)
    return (rows[:, None] * dim_beta + np.arange(dim_beta, dtype=np.int64)[None, :]).reshape(-1)


def _pick_rows(dim_alpha, k, seed):
    rng = np.random.default_rng(seed)
    inner = rng.choice(np.arange(1, dim_alpha - 1), k - 2, replace=False)
    return np.sort(np.concatenate([[0, dim_alpha - 1], inner]))


# each full-size workload runs with the unfactored evaluation and with the
# spin-factorized tables (factor tables, alpha lists, images; for the
# Hubbard sector the rows kernel), the configuration the benchmark times
@pytest.fixture(scope="module", params=[False, True], ids=["plain", "factored"])
def mol28(dev, request):
    api = _api()
    h1, h2 = synth.molecular_spin_integrals(14, seed=2001)
    G = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)).group()
    sp = api.Space.sector(14, 7, 7)
    if request.param:
        G.factor(sp)
    osp = ospace.SectorSpace(14, 7, 7)
    op = ojw.jw_sum(h1, h2)
    assert sp.dim == 11_778_624 and op.n_terms == 55_371
    return G, sp, osp, op, native.prepare(op, osp)


def test_28q_whole_rows_dense_state(dev, mol28):
    api = _api()
    G, sp, osp, op, prep = mol28
    rows = _pick_rows(osp.dim_alpha, 64, seed=28)
    tgt = _row_targets(rows, osp.dim_beta)
    tsel = torch.from_numpy(tgt).to(dev)
    psi = synth.random_state(sp.dim, seed=2101)
    print(f"[28q rows] {len(rows)} rows, {len(tgt)} targets, complex128", flush=True)
    ref, _ = native.apply_targets(op, osp, psi, tgt, prepared=prep)
    tpsi = torch.from_numpy(psi).to(dev)
    got = api.apply_pauli_sum(G, sp, tpsi)[tsel].cpu().numpy()
    assert rel_err(got, ref) < 1e-12
    for r in range(len(rows)):  # every row on its own, not only the sum over rows
        sl = slice(r * osp.dim_beta, (r + 1) * osp.dim_beta)
        assert rel_err(got[sl], ref[sl]) < 1e-12, f"row {rows[r]}"
    e_rows, e_rows_ref = np.vdot(psi[tgt], got), np.vdot(psi[tgt], ref)
    assert abs(e_rows - e_rows_ref) < 1e-12 * abs(e_rows_ref)

    print("[28q rows] complex64", flush=True)
    psi32 = psi.astype(np.complex64)
    ref32, _ = native.apply_targets(op, osp, psi32, tgt, prepared=prep)
    t32 = torch.from_numpy(psi32).to(dev)
    out32 = api.apply_pauli_sum(G, sp, t32)
    got32 = out32[tsel].cpu().numpy().astype(np.complex128)
    assert rel_err(got32, ref32) < 1e-6
    # the fused energy pass stores exactly what the plain apply stores
    fused = torch.empty_like(t32)
    api.expval(G, sp, t32, out=fused)
    assert torch.equal(torch.view_as_real(fused), torch.view_as_real(out32))


def _sparse_state(dim_alpha, dim_beta, n_rows, n_single, seed):
    rng = np.random.default_rng(seed)
    rows = rng.choice(dim_alpha, n_rows, replace=False)
    support = set(_row_targets(rows, dim_beta).tolist())
    support.update(rng.choice(dim_alpha * dim_beta, n_single, replace=False).tolist())
    support = np.array(sorted(support), dtype=np.int64)
    psi = np.zeros(dim_alpha * dim_beta, np.complex128)
    v = rng.standard_normal(len(support)) + 1j * rng.standard_normal(len(support))
    psi[support] = v / np.linalg.norm(v)
    return psi, support


def test_28q_sparse_support_whole_vector_and_energy(dev, mol28):
    api = _api()
    G, sp, osp, op, prep = mol28
    psi, support = _sparse_state(osp.dim_alpha, osp.dim_beta, 8, 500, seed=2801)
    for dtype, tol in ((torch.complex128, 1e-12), (torch.complex64, 1e-6)):
        print(f"[28q sparse] {len(support)} sources, whole vector, {dtype}", flush=True)
        src = psi.astype(np.complex64) if dtype == torch.complex64 else psi
        ref, _ = native.apply_scatter(op, osp, src, sources=support, prepared=prep)
        tpsi = torch.from_numpy(src).to(dev)
        out = torch.empty_like(tpsi)
        e = api.expval(G, sp, tpsi, out=out).cpu().numpy()
        got = out.cpu().numpy().astype(np.complex128)
        assert rel_err(got, ref) < tol
        e_ref = np.vdot(src.astype(np.complex128), ref)
        n_ref = np.vdot(src.astype(np.complex128), src.astype(np.complex128)).real
        if dtype == torch.complex128:
            assert abs(e[0] - e_ref.real) < 1e-12 * abs(e_ref)
        else:
            assert abs(e[0] - e_ref.real) < 1e-8
        assert abs(e[1] - e_ref.imag) < 1e-12 * abs(e_ref)
        assert abs(e[2] - n_ref) < 1e-13


def test_28q_hermiticity_dense_states(dev, mol28):
    """<phi|H psi> = conj(<psi|H phi>) over the whole dense vectors."""
    api = _api()
    G, sp, _, _, _ = mol28
    psi = torch.from_numpy(synth.random_state(sp.dim, seed=2101)).to(dev)
    phi = torch.from_numpy(synth.random_state(sp.dim, seed=2102)).to(dev)
    lhs = torch.vdot(phi, api.apply_pauli_sum(G, sp, psi)).item()
    rhs = torch.vdot(psi, api.apply_pauli_sum(G, sp, phi)).item().conjugate()
    assert abs(lhs - rhs) < 1e-11 * max(1.0, abs(lhs))


def _eighth(dim_alpha, r):
    return r * dim_alpha // 8, (r + 1) * dim_alpha // 8


def test_28q_one_eighth_row_share(dev, mol28):
    """One device's share of an eight-way split of the target alpha rows, in
    complex64 as the benchmark runs: bit-identical to the same rows of the
    whole-sector apply, four of its rows against the oracle, and the eight
    shares' energy sums adding up to the whole-sector energy."""
    api = _api()
    G, sp, osp, op, prep = mol28
    psi32 = synth.random_state(sp.dim, seed=2103).astype(np.complex64)
    t32 = torch.from_numpy(psi32).to(dev)
    whole = api.apply_pauli_sum(G, sp, t32)
    a0, a1 = _eighth(osp.dim_alpha, 3)
    print(f"[28q share] rows [{a0}, {a1}) of {osp.dim_alpha}, complex64", flush=True)
    share = api.apply_pauli_sum_rows(G, sp, t32, a0, a1)
    db = osp.dim_beta
    assert torch.equal(torch.view_as_real(share), torch.view_as_real(whole[a0 * db:a1 * db]))
    rows = np.array([a0, a0 + 17, a1 - 40, a1 - 1])
    ref, _ = native.apply_targets(op, osp, psi32, _row_targets(rows, db), prepared=prep)
    sel = torch.from_numpy(_row_targets(rows - a0, db)).to(dev)
    assert rel_err(share[sel].cpu().numpy().astype(np.complex128), ref) < 1e-6
    e_whole = api.expval(G, sp, t32).cpu().numpy()
    e_sum = sum(api.expval_rows(G, sp, t32, *_eighth(osp.dim_alpha, r)).cpu().numpy() for r in range(8))
    assert np.all(np.abs(e_sum - e_whole) < 1e-12 * max(1.0, abs(e_whole[0]))), (e_sum, e_whole)


@pytest.fixture(scope="module", params=[False, True], ids=["plain", "factored"])
def hub32(dev, request):
    api = _api()
    h1, h2 = synth.hubbard_spin_integrals(4, 4)
    G = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)).group()
    sp = api.Space.sector(16, 8, 8)
    if request.param:
        G.factor(sp)
    osp = ospace.SectorSpace(16, 8, 8)
    op = ojw.jw_sum(h1, h2)
    assert sp.dim == 165_636_900
    return G, sp, osp, op, native.prepare(op, osp)


def test_32q_hubbard_whole_rows(dev, hub32):
    api = _api()
    G, sp, osp, op, prep = hub32
    rows = _pick_rows(osp.dim_alpha, 16, seed=32)
    tgt = _row_targets(rows, osp.dim_beta)
    tsel = torch.from_numpy(tgt).to(dev)
    psi32 = synth.random_state(sp.dim, seed=4101).astype(np.complex64)
    ref, _ = native.apply_targets(op, osp, psi32, tgt, prepared=prep)
    print(f"[32q rows] {len(rows)} rows, complex64", flush=True)
    t32 = torch.from_numpy(psi32).to(dev)
    got = api.apply_pauli_sum(G, sp, t32)[tsel].cpu().numpy().astype(np.complex128)
    assert rel_err(got, ref) < 1e-6
    print("[32q rows] complex128", flush=True)
    t64 = t32.to(torch.complex128)
    del t32
    got64 = api.apply_pauli_sum(G, sp, t64)[tsel].cpu().numpy()
    assert rel_err(got64, ref) < 1e-12
    for r in range(len(rows)):
        sl = slice(r * osp.dim_beta, (r + 1) * osp.dim_beta)
        assert rel_err(got64[sl], ref[sl]) < 1e-12, f"row {rows[r]}"


def test_32q_hubbard_sparse_support_whole_vector(dev, hub32):
    api = _api()
    G, sp, osp, op, prep = hub32
    psi, support = _sparse_state(osp.dim_alpha, osp.dim_beta, 4, 2000, seed=3201)
    print(f"[32q sparse] {len(support)} sources, whole vector, complex64", flush=True)
    psi32 = psi.astype(np.complex64)
    del psi
    ref, _ = native.apply_scatter(op, osp, psi32, sources=support, threads=1, prepared=prep)
    t32 = torch.from_numpy(psi32).to(dev)
    out = torch.empty_like(t32)
    e = api.expval(G, sp, t32, out=out).cpu().numpy()
    got = out.cpu().numpy()
    del out
    assert rel_err(got.astype(np.complex128), ref) < 1e-6
    e_ref = np.vdot(psi32.astype(np.complex128), ref)
    assert abs(e[0] - e_ref.real) < 1e-8


def test_32q_hubbard_one_eighth_row_share(dev, hub32):
    """One device's share of an eight-way row split of the 4x4 Hubbard
    sector (complex64): bit-identical to those rows of the whole apply."""
    api = _api()
    G, sp, osp, _, _ = hub32
    t32 = torch.from_numpy(synth.random_state(sp.dim, seed=4103).astype(np.complex64)).to(dev)
    a0, a1 = _eighth(osp.dim_alpha, 5)
    print(f"[32q share] rows [{a0}, {a1}) of {osp.dim_alpha}, complex64", flush=True)
    share = api.apply_pauli_sum_rows(G, sp, t32, a0, a1)
    whole = api.apply_pauli_sum(G, sp, t32)
    db = osp.dim_beta
    assert torch.equal(torch.view_as_real(share), torch.view_as_real(whole[a0 * db:a1 * db]))
