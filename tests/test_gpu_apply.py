"""GPU parity of the operator-state product and the fused energy.

Tolerances: the FP64 path (complex128 storage, float64 accumulation) must
match the oracle to 1e-12 in the relative 2-norm.  The complex64 path stores
amplitudes in FP32 but accumulates in float64; it is compared with the oracle
run on the same FP32-rounded input upcast to float64, so the only error left
is the final rounding of each output amplitude to FP32 (relative 2^-24 ~
6e-8 per component), bounded here by 1e-6.  Energies from the fused
reduction never round the gathered H psi, so on identical inputs they agree
with the oracle to float64 accumulation error (1e-10 relative bound)."""

import numpy as np
import pytest
import torch

import synth
from oracle import apply as oapply
from oracle import jw as ojw
from oracle import pauli as opauli
from oracle import space as ospace
from tests.conftest import rel_err

pytestmark = pytest.mark.gpu


def _api():
    from paper_2606_28952_amd import api

    return api


def _gpu_op(dev, op):
    """Letter-form oracle PauliSum -> canonical, grouped GPU operator."""
    api = _api()
    x, z = op.xz()
    s = api.PauliSum.create(op.n_qubits, x.reshape(-1), z.reshape(-1), op.coeff)
    s.canonicalize()
    return s.group()


def _random_op(n, m, seed, hermitian=False):
    letters, _ = synth.random_pauli_strings(m, n, seed)
    rng = np.random.default_rng(seed + 1)
    c = rng.standard_normal(m) + (0 if hermitian else 1j * rng.standard_normal(m))
    return opauli.PauliSum(n, letters, c.astype(np.complex128))


def _run(dev, grouped, space, psi, dtype):
    api = _api()
    t = torch.from_numpy(psi.astype(dtype)).to(dev)
    return api.apply_pauli_sum(grouped, space, t).cpu().numpy()


@pytest.mark.parametrize("n,m", [(1, 2), (2, 5), (5, 40), (8, 120), (10, 300), (11, 50)])
def test_full_space_random_operator(dev, n, m):
    api = _api()
    op = _random_op(n, m, seed=10 + n)
    psi = synth.random_state(1 << n, seed=20 + n)
    G = _gpu_op(dev, op)
    sp = api.Space.full(n)
    ref = oapply.apply_scatter(op, ospace.FullSpace(n), psi)
    assert rel_err(_run(dev, G, sp, psi, np.complex128), ref) < 1e-12
    psi32 = psi.astype(np.complex64)
    ref32 = oapply.apply_scatter(op, ospace.FullSpace(n), psi32.astype(np.complex128))
    assert rel_err(_run(dev, G, sp, psi32, np.complex64), ref32) < 1e-6


def test_twelve_qubit_molecular_full_and_sector(dev):
    api = _api()
    h1, h2 = synth.molecular_spin_integrals(6, seed=1001)
    H = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev))
    G = H.group()
    op = ojw.jw_sum(h1, h2)
    for space, ospace_, seed in [(api.Space.full(12), ospace.FullSpace(12), 1101),
                                 (api.Space.sector(6, 3, 3), ospace.SectorSpace(6, 3, 3), 1102)]:
        psi = synth.random_state(ospace_.dim, seed)
        ref = oapply.apply_scatter(op, ospace_, psi)
        out = _run(dev, G, space, psi, np.complex128)
        assert rel_err(out, ref) < 1e-12
        psi32 = psi.astype(np.complex64)
        ref32 = oapply.apply_scatter(op, ospace_, psi32.astype(np.complex128))
        assert rel_err(_run(dev, G, space, psi32, np.complex64), ref32) < 1e-6
        tpsi = torch.from_numpy(psi).to(dev)
        fused = torch.empty_like(tpsi)
        e = api.expval(G, space, tpsi, out=fused).cpu().numpy()
        # the fused pass stores exactly what the plain apply stores
        assert torch.equal(torch.view_as_real(fused), torch.view_as_real(api.apply_pauli_sum(G, space, tpsi)))
        e_ref = np.vdot(psi, ref)
        assert abs(e[0] - e_ref.real) < 1e-12 * abs(e_ref) and abs(e[1]) < 1e-12 * abs(e_ref)
        assert abs(e[2] - 1.0) < 1e-13
        e32 = api.expval(G, space, torch.from_numpy(psi32).to(dev)).cpu().numpy()
        e32_ref = np.vdot(psi32.astype(np.complex128), ref32)
        assert abs(e32[0] - e32_ref.real) < 1e-10 * abs(e32_ref)


def _sector_compatible_op(n_o, seed, m=400):
    """Random non-conserving operator on 2 n_o qubits whose strings mostly
    (~70%) flip an even number of orbitals in each spin half, so that a
    sector sees nonzero coupling."""
    n = 2 * n_o
    rng = np.random.default_rng(seed)
    letters, _ = synth.random_pauli_strings(m, n, seed=n_o + 7)
    for k in range(m):
        if rng.random() < 0.7:
            for half in (0, 1):
                cols = np.arange(half * n_o, (half + 1) * n_o)
                flips = cols[(letters[k, cols] == 1) | (letters[k, cols] == 2)]
                if len(flips) % 2 == 1:
                    letters[k, flips[0]] = 3
    coeff = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    return opauli.PauliSum(n, letters, coeff)


@pytest.mark.parametrize("n_o,na,nb", [(1, 0, 1), (1, 1, 1), (3, 1, 2), (4, 0, 4), (5, 2, 3), (9, 4, 5),
                                       (11, 5, 5), (12, 6, 6), (13, 6, 6), (15, 1, 7), (16, 1, 8)])
def test_sector_projection_random_operator(dev, n_o, na, nb):
    """Non-conserving random operators: the sector result is P H P psi.  The
    operators carry many strings with even X popcounts per spin so that the
    sector sees nonzero coupling; beta dimensions span 1 to 12,870 columns
    (several lanes per thread, ragged tails; rows of 6,435 and 12,870
    columns exceed LDS and are staged in tiles)."""
    api = _api()
    op = _sector_compatible_op(n_o, n_o * 31 + na)
    osp = ospace.SectorSpace(n_o, na, nb)
    G = _gpu_op(dev, op)
    sp = api.Space.sector(n_o, na, nb)
    psi = synth.random_state(osp.dim, seed=n_o + 100)
    if osp.dim <= 200_000:
        ref = oapply.apply_scatter(op, osp, psi)
        assert rel_err(_run(dev, G, sp, psi, np.complex128), ref) < 1e-12
    else:
        sel = np.random.default_rng(1).integers(0, osp.dim, 300)
        got = _run(dev, G, sp, psi, np.complex128)[sel]
        ref = oapply.apply_targets(op, osp, psi, sel)
        assert rel_err(got, ref) < 1e-12


@pytest.mark.parametrize("n_o,na,nb", [(17, 1, 1), (20, 1, 2), (24, 2, 1)])
def test_sector_above_sixteen_orbitals(dev, n_o, na, nb):
    """More than 16 orbitals: spin strings are ranked through the global
    rank tables (the kernel variants without LDS rank tables); both storage
    types, the plain apply and the fused energy, against the oracle."""
    api = _api()
    op = _sector_compatible_op(n_o, n_o * 17 + nb)
    osp = ospace.SectorSpace(n_o, na, nb)
    G = _gpu_op(dev, op)
    sp = api.Space.sector(n_o, na, nb)
    psi = synth.random_state(osp.dim, seed=n_o + 200)
    ref = oapply.apply_scatter(op, osp, psi)
    assert rel_err(_run(dev, G, sp, psi, np.complex128), ref) < 1e-12
    psi32 = psi.astype(np.complex64)
    ref32 = oapply.apply_scatter(op, osp, psi32.astype(np.complex128))
    assert rel_err(_run(dev, G, sp, psi32, np.complex64), ref32) < 1e-6
    for p, r, tol in ((psi, ref, 1e-12), (psi32.astype(np.complex128), ref32, 1e-10)):
        for dt in ((torch.complex128,) if tol == 1e-12 else (torch.complex64,)):
            e = api.expval(G, sp, torch.from_numpy(p).to(dev).to(dt)).cpu().numpy()
            e_ref = np.vdot(p, r)
            assert abs(e[0] - e_ref.real) < tol * max(1.0, abs(e_ref))
            assert abs(e[1] - e_ref.imag) < tol * max(1.0, abs(e_ref))


def test_batch_mixes_orbital_counts_above_and_below_sixteen(dev):
    """One launch over jobs with n_orb <= 16 and > 16 takes the global rank
    tables for all of them; each job still matches the oracle."""
    api = _api()
    specs = [(6, 3, 2, 61), (17, 1, 1, 62), (9, 4, 4, 63), (20, 2, 1, 64)]
    jobs, refs = [], []
    for n_o, na, nb, seed in specs:
        op = _sector_compatible_op(n_o, seed)
        osp = ospace.SectorSpace(n_o, na, nb)
        psi = synth.random_state(osp.dim, seed=seed + 1)
        t = torch.from_numpy(psi).to(dev)
        jobs.append((_gpu_op(dev, op), api.Space.sector(n_o, na, nb), t, torch.empty_like(t)))
        refs.append((psi, oapply.apply_scatter(op, osp, psi)))
    batch = api.Batch(jobs)
    energies = torch.zeros(3 * len(jobs), dtype=torch.float64, device=dev)
    batch.run(energies)
    torch.cuda.synchronize()
    e = energies.cpu().numpy().reshape(-1, 3)
    for k, ((_, _, _, out), (psi, ref)) in enumerate(zip(jobs, refs)):
        assert rel_err(out.cpu().numpy(), ref) < 1e-12, f"job {k}"
        e_ref = np.vdot(psi, ref)
        assert abs(e[k, 0] - e_ref.real) < 1e-12 * max(1.0, abs(e_ref)), f"job {k}"


def test_twenty_qubit_molecular_sector(dev):
    api = _api()
    h1, h2 = synth.molecular_spin_integrals(10, seed=4)
    H = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev))
    G = H.group()
    op = ojw.jw_sum(h1, h2)
    osp = ospace.SectorSpace(10, 5, 5)
    psi = synth.random_state(osp.dim, seed=5)
    ref = oapply.apply_scatter(op, osp, psi)
    sp = api.Space.sector(10, 5, 5)
    out = _run(dev, G, sp, psi, np.complex128)
    assert rel_err(out, ref) < 1e-12
    # a second spin sector of the same operator
    osp2 = ospace.SectorSpace(10, 4, 6)
    psi2 = synth.random_state(osp2.dim, seed=6)
    assert rel_err(_run(dev, G, api.Space.sector(10, 4, 6), psi2, np.complex128),
                   oapply.apply_scatter(op, osp2, psi2)) < 1e-12


def test_deterministic_and_edge_operators(dev):
    api = _api()
    h1, h2 = synth.molecular_spin_integrals(5, seed=9)
    G = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)).group()
    sp = api.Space.sector(5, 2, 3)
    psi = torch.from_numpy(synth.random_state(sp.dim, 3)).to(dev)
    a = api.apply_pauli_sum(G, sp, psi)
    b = api.apply_pauli_sum(G, sp, psi)
    assert torch.equal(a.view(torch.float64), b.view(torch.float64))
    # empty operator: zero output
    empty = api.PauliSum.create(10, np.zeros(0, np.uint64), np.zeros(0, np.uint64), np.zeros(0, np.complex128))
    empty.canonicalize()
    Ge = empty.group()
    out = api.apply_pauli_sum(Ge, sp, psi)
    assert torch.count_nonzero(out) == 0
    out_full = api.apply_pauli_sum(Ge, api.Space.full(10), torch.ones(1024, dtype=torch.complex64, device=dev))
    assert torch.count_nonzero(out_full) == 0
    # identity times a complex constant
    ident = api.PauliSum.create(10, np.zeros(1, np.uint64), np.zeros(1, np.uint64), np.array([0.5 - 2j]))
    ident.canonicalize()
    out = api.apply_pauli_sum(ident.group(), sp, psi)
    assert torch.allclose(out, (0.5 - 2j) * psi, rtol=0, atol=1e-15)


def test_argument_errors(dev):
    api = _api()
    from paper_2606_28952_amd._abi import PbsError

    h1, h2 = synth.molecular_spin_integrals(3, seed=1)
    G = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)).group()
    sp = api.Space.sector(3, 1, 1)
    psi = torch.zeros(sp.dim, dtype=torch.complex128, device=dev)
    with pytest.raises(PbsError, match="overlaps"):
        api.apply_pauli_sum(G, sp, psi, out=psi)
    with pytest.raises(PbsError, match="qubits"):
        api.apply_pauli_sum(G, api.Space.full(8), torch.zeros(256, dtype=torch.complex128, device=dev))
    with pytest.raises(PbsError, match="workspace"):
        work = torch.zeros(1, dtype=torch.float64, device=dev)
        api.expval(G, sp, psi, work=work)
    with pytest.raises(PbsError, match="overlaps"):
        api.expval(G, sp, psi, out=psi)
