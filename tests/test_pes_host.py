"""Host logic of the scan module (no GPU): the rotation generators' X/Z
masks against the oracle's independent conversion of their letter form, and
the scan summary."""

import numpy as np
import pytest

import synth
from oracle import pauli as opauli
from paper_2606_28952_amd import pes


@pytest.mark.parametrize("n_orb,na,nb,count", [(6, 3, 3, 200), (3, 2, 1, 40), (12, 6, 6, 200), (14, 7, 7, 400)])
def test_excitation_masks_match_letters(n_orb, na, nb, count):
    letters = synth.excitation_generators(n_orb, na, nb, count)
    x, z = synth.excitation_masks(n_orb, na, nb, count)
    xo, zo = opauli.letters_to_xz(letters)
    assert x.dtype == np.uint64 and z.dtype == np.uint64
    np.testing.assert_array_equal(x, xo[:, 0])
    np.testing.assert_array_equal(z, zo[:, 0])


def test_excitation_generators_are_hermitian_imaginary_strings():
    # odd number of Y letters: i P is real, so the rotations keep a real state real
    gens = synth.excitation_generators(6, 3, 3, 200)
    assert len(gens) == 9 + 9 + 9 + 9 + 81  # singles, then same-spin and opposite-spin doubles
    assert all(int((g == 2).sum()) == 1 for g in gens)
    x, z = synth.excitation_masks(6, 3, 3, 200)
    assert len(set(x.tolist())) == len(x)  # distinct qubit sets
    assert all(bin(int(a) & int(b)).count("1") == 1 for a, b in zip(x, z))  # one Y each


def test_scan_rejects_mismatched_masks():
    with pytest.raises(ValueError):
        pes.scan(None, [], 2, np.zeros(3, np.uint64), np.zeros(2, np.uint64), 0)


def test_summary_totals():
    recs = [dict(iters_cold=10, evals_cold=12, iters_warm=6, evals_warm=8, start="network", E_warm=-1.0,
                 E_cold=-1.0 + 1e-12),
            dict(iters_cold=20, evals_cold=22, iters_warm=20, evals_warm=22, start="cold", E_warm=-2.0, E_cold=-2.0)]
    s = pes.summary(recs)
    assert (s["iters_cold"], s["iters_warm"], s["evals_cold"], s["evals_warm"]) == (30, 26, 34, 30)
    assert s["network_starts"] == 1
    assert s["min_E_warm_minus_cold"] < 0 and s["max_E_warm_minus_cold"] == 0.0
