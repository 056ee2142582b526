"""Host logic of the benchmark (no GPU): the combinatorial count of
connected groups per target (the roofline's algorithmic bytes) against brute
force over every target of small sectors, the kernel-source hash, and the
refusal of more than one GPU."""

import os
import subprocess
import sys

import numpy as np
import pytest

import bench
import synth
from oracle import jw as ojw
from oracle import pauli as opauli
from oracle import space as ospace

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _brute_connected(xg, sizes, osp):
    """Average over the sector's targets of the number of groups (and of
    their strings) whose source t ^ X lies in the sector."""
    n = osp.n_orb
    ta = np.asarray(osp.alpha, dtype=np.int64)
    tb = np.asarray(osp.beta, dtype=np.int64)
    in_a, in_b = set(ta.tolist()), set(tb.tolist())
    groups = strings = 0
    for x, w in zip(xg.tolist(), sizes.tolist()):
        xa, xb = x & ((1 << n) - 1), x >> n
        ca = sum(1 for t in ta.tolist() if (t ^ xa) in in_a)
        cb = sum(1 for t in tb.tolist() if (t ^ xb) in in_b)
        groups += ca * cb
        strings += ca * cb * w
    d = len(ta) * len(tb)
    return groups / d, strings / d


@pytest.mark.parametrize("n_orb,na,nb,seed", [(4, 2, 2, 5), (5, 3, 1, 6), (6, 2, 3, 7)])
def test_connected_groups_match_brute_force(n_orb, na, nb, seed):
    h1, h2 = synth.molecular_spin_integrals(n_orb, seed)
    x, z, c = ojw.jw_hamiltonian(h1, h2)
    xg, off, _, _ = opauli.group_by_x(x, z, c)
    sizes = np.diff(off.astype(np.int64))
    osp = ospace.SectorSpace(n_orb, na, nb)
    want_g, want_s = _brute_connected(xg, sizes, osp)
    assert bench._connected_groups(xg, n_orb, na, nb) == pytest.approx(want_g, rel=1e-12)
    assert bench._connected_groups(xg, n_orb, na, nb, weights=sizes) == pytest.approx(want_s, rel=1e-12)


def test_source_hash_is_stable_and_short():
    h = bench._source_hash()
    assert h == bench._source_hash() and len(h) == 16 and int(h, 16) >= 0


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
