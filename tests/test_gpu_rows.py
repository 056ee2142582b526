"""Target-row shares of the sector apply (Eq. reverse_sum, Eq.
sreverse_sum: every target amplitude is evaluated on its own, so the alpha
rows of a sector split into independent shares that each need the whole
state and no reduction).

Each share runs the whole-sector kernels on its rows only, so the shares
concatenated must equal the whole-sector output bit for bit (and hence
meet the oracle's bars), for the sector kernel (unfactored and factored)
and for the rows kernel (long Hubbard rows); the shares' energy sums add up
to the whole-sector energy within float64 accumulation error.  Uneven and
empty shares, a single-row share and the last row are covered, as are the
refusals of a full space, a range past the sector and an overlapping
output."""

import numpy as np
import pytest
import torch

import synth
from oracle import apply as oapply
from oracle import jw as ojw
from oracle import space as ospace
from tests.conftest import rel_err

pytestmark = pytest.mark.gpu


def _api():
    from paper_2606_28952_amd import api

    return api


def _bounds(dim_alpha):
    """Uneven shares: an empty one, a single row, a ragged middle, the rest."""
    cuts = sorted({0, 0, 1, max(1, dim_alpha // 3), max(1, (2 * dim_alpha) // 3 + 1), dim_alpha})
    cuts = [c for c in cuts if c <= dim_alpha]
    return [(0, 0)] + list(zip(cuts[:-1], cuts[1:])) + [(dim_alpha, dim_alpha)]


def _check_shares(api, G, sp, psi, whole, e_whole):
    dim_alpha, dim_beta = sp.shape()[3], sp.shape()[4]
    parts, e_sum = [], np.zeros(3)
    for a0, a1 in _bounds(dim_alpha):
        print(f"[rows] share [{a0}, {a1}) of {dim_alpha}, dtype {psi.dtype}", flush=True)
        part = api.apply_pauli_sum_rows(G, sp, psi, a0, a1)
        assert part.numel() == (a1 - a0) * dim_beta
        parts.append(part)
        out = torch.empty_like(part)
        e = api.expval_rows(G, sp, psi, a0, a1, out=out).cpu().numpy()
        assert torch.equal(torch.view_as_real(out), torch.view_as_real(part))
        # the energy alone (no stored product) gives the same bits, also with
        # a workspace sized for the share only
        assert np.array_equal(api.expval_rows(G, sp, psi, a0, a1).cpu().numpy(), e)
        chunks = (dim_beta + 511) // 512
        small = torch.empty(max(1, (a1 - a0) * chunks * 3), dtype=torch.float64, device=psi.device)
        assert np.array_equal(api.expval_rows(G, sp, psi, a0, a1, work=small).cpu().numpy(), e)
        e_sum += e
    got = torch.cat(parts)
    assert torch.equal(torch.view_as_real(got), torch.view_as_real(whole))
    scale = max(1.0, float(np.abs(e_whole[:2]).max()))
    assert np.all(np.abs(e_sum - e_whole) < 1e-12 * scale), (e_sum, e_whole)


CASES = [(6, 3, 3, 1001, False), (6, 3, 3, 1001, True), (8, 3, 5, 41, True), (9, 5, 4, 44, False)]


@pytest.mark.parametrize("n_o,na,nb,seed,factored", CASES)
def test_molecular_shares_equal_whole_sector(dev, n_o, na, nb, seed, factored):
    api = _api()
    h1, h2 = synth.molecular_spin_integrals(n_o, seed)
    G = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)).group()
    sp = api.Space.sector(n_o, na, nb)
    if factored:
        G.factor(sp)
    psi_np = synth.random_state(sp.dim, seed + 3)
    ref = oapply.apply_scatter(ojw.jw_sum(h1, h2), ospace.SectorSpace(n_o, na, nb), psi_np)
    for cdt in (torch.complex128, torch.complex64):
        psi = torch.from_numpy(psi_np).to(dev).to(cdt)
        whole = api.apply_pauli_sum(G, sp, psi)
        if cdt == torch.complex128:
            assert rel_err(whole.cpu().numpy(), ref) < 1e-12
        _check_shares(api, G, sp, psi, whole, api.expval(G, sp, psi).cpu().numpy())


def test_hubbard_rows_kernel_shares(dev):
    """Long rows (6,435 beta strings) on the factored rows kernel."""
    api = _api()
    h1, h2 = synth.hubbard_spin_integrals(3, 5)
    n_o, na, nb = 15, 2, 7
    G = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)).group()
    sp = api.Space.sector(n_o, na, nb)
    G.factor(sp)
    psi_np = synth.random_state(sp.dim, 72)
    ref = oapply.apply_scatter(ojw.jw_sum(h1, h2), ospace.SectorSpace(n_o, na, nb), psi_np)
    for cdt in (torch.complex128, torch.complex64):
        psi = torch.from_numpy(psi_np).to(dev).to(cdt)
        whole = api.apply_pauli_sum(G, sp, psi)
        if cdt == torch.complex128:
            assert rel_err(whole.cpu().numpy(), ref) < 1e-12
        _check_shares(api, G, sp, psi, whole, api.expval(G, sp, psi).cpu().numpy())


def test_row_range_refusals(dev):
    api = _api()
    from paper_2606_28952_amd._abi import PbsError

    h1, h2 = synth.molecular_spin_integrals(4, 5)
    G = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)).group()
    sp = api.Space.sector(4, 2, 2)  # 6 x 6
    psi = torch.from_numpy(synth.random_state(sp.dim, 9)).to(dev)
    with pytest.raises(PbsError, match="outside"):
        api.apply_pauli_sum_rows(G, sp, psi, 2, 7)
    with pytest.raises(PbsError, match="outside"):
        api.apply_pauli_sum_rows(G, sp, psi, 4, 3)
    with pytest.raises(PbsError, match="overlaps"):
        api.apply_pauli_sum_rows(G, sp, psi, 0, 2, out=psi[6:18])
    with pytest.raises(PbsError, match="workspace"):  # 3 rows x 1 chunk x 3 doubles needed
        api.expval_rows(G, sp, psi, 1, 4, work=torch.empty(8, dtype=torch.float64, device=dev))
    full = api.Space.full(8)
    psi_f = torch.from_numpy(synth.random_state(full.dim, 9)).to(dev)
    with pytest.raises(PbsError, match="sector"):
        api.expval_rows(G, full, psi_f, 0, 1)
