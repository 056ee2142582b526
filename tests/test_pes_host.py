"""Host logic of the scan driver (no GPU): letter strings to X/Z masks
against the oracle's independent conversion, and the scan summary."""

import numpy as np
import pytest

import synth
from oracle import pauli as opauli
from paper_2606_28952_amd import pes


def test_letters_to_masks_matches_oracle():
    rng = np.random.default_rng(0)
    for n in (1, 7, 24, 64):
        letters = rng.integers(0, 4, size=(50, n)).astype(np.uint8)
        x, z = pes.letters_to_masks(letters)
        xo, zo = opauli.letters_to_xz(letters)
        np.testing.assert_array_equal(x, xo[:, 0])
        np.testing.assert_array_equal(z, zo[:, 0])
    with pytest.raises(ValueError):
        pes.letters_to_masks(np.zeros((1, 65), np.uint8))


def test_excitation_generators_are_hermitian_imaginary_strings():
    # odd number of Y letters: i P is real, so the rotations keep a real state real
    gens = synth.excitation_generators(6, 3, 3, 200)
    assert len(gens) == 9 + 9 + 9 + 9 + 81  # singles, then same-spin and opposite-spin doubles
    assert all(int((g == 2).sum()) == 1 for g in gens)
    x, _ = pes.letters_to_masks(gens)
    assert len(set(x.tolist())) == len(x)  # distinct qubit sets


def test_summary_totals():
    recs = [dict(iters_cold=10, evals_cold=12, iters_warm=6, evals_warm=8, start="network", E_warm=-1.0,
                 E_cold=-1.0 + 1e-12),
            dict(iters_cold=20, evals_cold=22, iters_warm=20, evals_warm=22, start="cold", E_warm=-2.0, E_cold=-2.0)]
    s = pes.summary(recs)
    assert (s["iters_cold"], s["iters_warm"], s["evals_cold"], s["evals_warm"]) == (30, 26, 34, 30)
    assert s["network_starts"] == 1
    assert s["min_E_warm_minus_cold"] < 0 and s["max_E_warm_minus_cold"] == 0.0
