"""GPU tests of the variational loop and the learned warm start: L-BFGS on
the device energy reaches a stationary point whose energy the oracle
confirms, and on a potential-energy scan the network-started runs need
fewer iterations than cold starts at the same final energies, with the
cold start taking over when the network has nothing to offer."""

import numpy as np
import pytest
import torch

import synth
from oracle import apply as oapply
from oracle import jw as ojw
from oracle import vqe as ovqe

pytestmark = pytest.mark.gpu


def _mods():
    from paper_2606_28952_amd import api, pes

    return api, pes


def _ref(n_orb, na, nb):
    return ((1 << na) - 1) | (((1 << nb) - 1) << n_orb)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_minimize_reaches_a_confirmed_stationary_point(dev, dtype):
    api, pes = _mods()
    n_orb, na, nb = 3, 2, 1
    h1, h2 = synth.pes_integrals(n_orb, 0.4)
    G = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)).group()
    gens = synth.excitation_generators(n_orb, na, nb, 40)
    x, z = synth.excitation_masks(n_orb, na, nb, 40)
    ref = _ref(n_orb, na, nb)
    v = api.VQE(G, n_orb, x, z, ref, dtype=dtype)
    g_tol = 1e-6 if dtype == torch.complex128 else 2e-3
    th, e, it, ev, why = v.minimize(np.zeros(len(x)), g_tol=g_tol)
    assert why == "gradient" and 0 < it <= ev
    e2, g = v.energy_grad(th)
    assert np.abs(g).max() <= g_tol
    op = ojw.jw_sum(h1, h2)
    e_or = ovqe.energy(op, gens, th, ref)
    tol = 1e-11 if dtype == torch.complex128 else 1e-5
    assert abs(e - e_or) < tol * abs(e_or) and abs(e2 - e_or) < tol * abs(e_or)
    H = oapply.dense_matrix(op)
    assert np.linalg.eigvalsh(H)[0] - 1e-9 <= e_or < H[ref, ref].real


def _scan(dev, n_orb, na, nb, n_rot, n_geo, **kw):
    api, pes = _mods()
    x, z = synth.excitation_masks(n_orb, na, nb, n_rot)
    return pes.scan(lambda r: synth.pes_integrals(n_orb, r), np.linspace(0, 1, n_geo), n_orb, x, z,
                    _ref(n_orb, na, nb), mlp_params=synth.mlp_init(256, len(x), seed=2), **kw)


def test_warm_start_saves_iterations_at_equal_energy(dev):
    _, pes = _mods()
    recs = _scan(dev, 6, 3, 3, 117, 12)
    s = pes.summary(recs)
    assert s["network_starts"] >= 10
    assert s["iters_warm"] < 0.85 * s["iters_cold"], s
    assert s["evals_warm"] < 0.9 * s["evals_cold"], s
    assert max(abs(r["E_warm"] - r["E_cold"]) for r in recs) < 1e-8
    assert all(r["stop_warm"] == "gradient" and r["stop_cold"] == "gradient" for r in recs)
    # the network's guess is already close: far below the reference energy
    for r in recs[2:]:
        assert r["E_start"] - r["E_warm"] < 0.05 * (r["E_ref"] - r["E_warm"])


def test_untrained_network_falls_back_to_cold_start(dev):
    recs = _scan(dev, 4, 2, 2, 26, 4, min_train=100)
    for r in recs:
        assert r["start"] == "cold"
        assert (r["iters_warm"], r["E_warm"]) == (r["iters_cold"], r["E_cold"])


def test_poor_prediction_falls_back_to_cold_start(dev):
    api, pes = _mods()
    n_orb, na, nb = 4, 2, 2
    x, z = synth.excitation_masks(n_orb, na, nb, 26)
    p = synth.mlp_init(256, len(x), seed=3)
    p[-len(x):] = 2.0  # output bias: every angle near 2 rad, far from the minimum
    recs = pes.scan(lambda r: synth.pes_integrals(n_orb, r), [0.0, 0.5], n_orb, x, z, _ref(n_orb, na, nb),
                    mlp_params=p, train_steps=0)
    assert recs[1]["start"] == "cold"
    assert recs[1]["E_warm"] == recs[1]["E_cold"]
