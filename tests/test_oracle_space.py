"""Pins of the oracle's configuration spaces: printed determinant counts,
closed-form dimensions and an exhaustive rank/unrank bijection."""

from math import comb

import numpy as np
import pytest

from oracle import space
from tests.conftest import golden_rows


def test_fcidim_matches_printed_table():
    for system, basis, ne, no, det in golden_rows("fcidim_table.txt"):
        ne, no = int(ne), int(no)
        dim = comb(no, ne // 2) * comb(no, ne - ne // 2)   # Eq. fcidim
        assert float("%.2g" % dim) == float(det), system


@pytest.mark.parametrize("n_o,na,nb,dim", [(6, 3, 3, 400), (14, 7, 7, 11_778_624), (16, 8, 8, 165_636_900),
                                           (10, 5, 5, 63_504), (12, 6, 6, 853_776)])
def test_sector_dimensions(n_o, na, nb, dim):
    assert comb(n_o, na) * comb(n_o, nb) == dim
    if dim < 2_000_000:
        assert space.SectorSpace(n_o, na, nb).dim == dim


@pytest.mark.parametrize("n_o", range(1, 13))
def test_spin_strings_exhaustive(n_o):
    for n in range(0, n_o + 1):
        s = space.spin_strings(n_o, n)
        want = [w for w in range(1 << n_o) if bin(w).count("1") == n]
        assert s.tolist() == want


@pytest.mark.parametrize("n_o,na,nb", [(4, 2, 2), (5, 2, 3), (6, 3, 3), (6, 0, 6), (7, 3, 2)])
def test_sector_index_bijection(n_o, na, nb):
    sp = space.SectorSpace(n_o, na, nb)
    basis = sp.basis()
    np.testing.assert_array_equal(sp.index_of(basis), np.arange(sp.dim))
    # every other pattern of 2 n_o bits is outside
    allbits = np.arange(1 << (2 * n_o), dtype=np.uint64)
    idx = sp.index_of(allbits)
    inside = (np.bitwise_count(allbits & np.uint64((1 << n_o) - 1)) == na) & \
             (np.bitwise_count(allbits >> np.uint64(n_o)) == nb)
    assert ((idx >= 0) == inside).all()
    # alpha-major layout
    ia, ib = np.divmod(np.arange(sp.dim), sp.dim_beta)
    np.testing.assert_array_equal(basis & np.uint64((1 << n_o) - 1), sp.alpha[ia])
    np.testing.assert_array_equal(basis >> np.uint64(n_o), sp.beta[ib])


def test_full_space_identity():
    sp = space.FullSpace(5)
    np.testing.assert_array_equal(sp.index_of(sp.basis()), np.arange(32))
    assert sp.index_of(np.array([32], np.uint64))[0] == -1
