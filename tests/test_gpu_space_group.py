"""GPU parity of the sector indexing (rank/unrank) and of the X-mask
grouping, bit-exact against the oracle."""

import numpy as np
import pytest
import torch

import synth
from oracle import jw as ojw
from oracle import pauli as opauli
from oracle import space as ospace

pytestmark = pytest.mark.gpu


def _api():
    from paper_2606_28952_amd import api

    return api


@pytest.mark.parametrize("n_o,na,nb", [(1, 0, 1), (1, 1, 1), (4, 2, 2), (6, 3, 3), (7, 0, 7), (9, 4, 2),
                                       (12, 6, 6), (14, 7, 7), (16, 8, 8), (20, 3, 2), (32, 2, 1)])
def test_sector_rank_unrank(dev, n_o, na, nb):
    api = _api()
    sp = api.Space.sector(n_o, na, nb)
    osp = ospace.SectorSpace(n_o, na, nb)
    assert sp.dim == osp.dim
    assert sp.shape() == (n_o, na, nb, osp.dim_alpha, osp.dim_beta)
    if osp.dim <= 20_000_000:
        idx = torch.arange(osp.dim, dtype=torch.int64, device=dev)
        want = osp.basis()
    else:
        sel = np.random.default_rng(n_o).integers(0, osp.dim, 1_000_000)
        idx = torch.from_numpy(sel).to(dev)
        ia, ib = np.divmod(sel, osp.dim_beta)
        want = osp.alpha[ia] | (osp.beta[ib] << np.uint64(n_o))
    bits = sp.unrank(idx)
    np.testing.assert_array_equal(bits.cpu().numpy().view(np.uint64), want)
    back = sp.rank(bits)
    np.testing.assert_array_equal(back.cpu().numpy(), idx.cpu().numpy())


@pytest.mark.parametrize("n_o,na,nb", [(4, 2, 2), (5, 1, 3), (8, 4, 4)])
def test_sector_rank_outside(dev, n_o, na, nb):
    api = _api()
    sp = api.Space.sector(n_o, na, nb)
    osp = ospace.SectorSpace(n_o, na, nb)
    allbits = np.arange(1 << (2 * n_o), dtype=np.uint64)
    extra = np.array([1 << (2 * n_o), (1 << 63) | 3], dtype=np.uint64)   # bits above the sector
    probe = np.concatenate([allbits, extra])
    got = sp.rank(torch.from_numpy(probe.view(np.int64)).to(dev)).cpu().numpy()
    np.testing.assert_array_equal(got, osp.index_of(probe))


def test_unrank_out_of_range(dev):
    api = _api()
    sp = api.Space.sector(6, 3, 3)
    bits = sp.unrank(torch.tensor([-1, 400, 399, 0], dtype=torch.int64, device=dev)).cpu().numpy().view(np.uint64)
    assert bits[0] == np.uint64(2 ** 64 - 1) and bits[1] == np.uint64(2 ** 64 - 1)
    osp = ospace.SectorSpace(6, 3, 3)
    assert bits[2] == osp.basis()[399] and bits[3] == osp.basis()[0]


def test_full_space_rank_unrank(dev):
    api = _api()
    sp = api.Space.full(10)
    probe = torch.tensor([0, 5, 1023, 1024, -1], dtype=torch.int64, device=dev)
    np.testing.assert_array_equal(sp.rank(probe).cpu().numpy(), [0, 5, 1023, -1, -1])
    np.testing.assert_array_equal(sp.unrank(torch.tensor([3, 1024], device=dev)).cpu().numpy().view(np.uint64),
                                  [3, 2 ** 64 - 1])


@pytest.mark.parametrize("case", ["mol6", "mol10", "tfim", "hubbard"])
def test_group_by_xmask_bit_exact(dev, case):
    api = _api()
    if case.startswith("mol"):
        h1, h2 = synth.molecular_spin_integrals(int(case[3:]), seed=5)
        x, z, c = ojw.jw_hamiltonian(h1, h2)
        nq = h1.shape[0]
    elif case == "hubbard":
        h1, h2 = synth.hubbard_spin_integrals(4, 4)
        x, z, c = ojw.jw_hamiltonian(h1, h2)
        nq = 32
    else:
        op = opauli.PauliSum.from_text(synth.tfim_terms(20))
        x, z, c = opauli.canonical_arrays(op)
        nq = 20
    s = api.PauliSum.create(nq, x.reshape(-1), z.reshape(-1), c)
    s.canonicalize()
    g = s.group()
    gx, goff, gz, gc = g.read()
    rx, roff, rz, rc = opauli.group_by_x(x, z, c)
    np.testing.assert_array_equal(gx, rx)
    np.testing.assert_array_equal(goff, roff)
    np.testing.assert_array_equal(gz, rz)
    assert gc.tobytes() == rc.astype(np.complex128).tobytes()
    if case == "tfim":
        assert g.n_groups == 21 and len(gc) == 39
    if case == "hubbard":
        assert g.n_groups == 65


def test_group_requires_canonical(dev):
    api = _api()
    from paper_2606_28952_amd._abi import PbsError

    s = api.PauliSum.create(4, np.array([1, 1], np.uint64), np.array([0, 0], np.uint64), np.array([1.0, 2.0]))
    with pytest.raises(PbsError, match="canonical"):
        s.group()
