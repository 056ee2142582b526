"""Rank structure of the per-group phase matrices of a Jordan-Wigner
molecular Hamiltonian (Section 2.4, the tensor-rank factorization behind
Algorithm 2 and Table svd_rank_dist).

For each X-mask group g, M^(g)[mu, nu] sums the XZ-form coefficients of the
group's terms with alpha Z-mask mu and beta Z-mask nu, so that the group's
phase sum at s is a(s_alpha)^T M^(g) b(s_beta) with a, b vectors of signs.
The spin-factorized evaluation relies on these ranks being small: the
diagonal group has rank n_o + 2, the 2 C(n_o, 2) same-spin hopping groups
rank 2, and every other group rank 1.  The kernels use the rank-1 structure
of the opposite-spin double groups directly (alpha factor folded per
workgroup, beta parity cached per move)."""

import collections
from math import comb

import numpy as np
import pytest

import synth
from oracle import jw as ojw
from oracle import pauli as opauli


def _group_ranks(n_o, seed):
    h1, h2 = synth.molecular_spin_integrals(n_o, seed=seed)
    op = ojw.jw_sum(h1, h2)
    x, z = op.xz()
    xs, off, zk, ck = opauli.group_by_x(x, z, op.coeff)
    mask = (1 << n_o) - 1
    out = collections.Counter()
    for g in range(len(xs)):
        X = int(xs[g])
        zz = zk[off[g]:off[g + 1]].astype(np.int64)
        cc = ck[off[g]:off[g + 1]]
        za, zb = zz & mask, zz >> n_o
        rows = {v: i for i, v in enumerate(sorted(set(za.tolist())))}
        cols = {v: i for i, v in enumerate(sorted(set(zb.tolist())))}
        M = np.zeros((len(rows), len(cols)), complex)
        for a, b, c in zip(za.tolist(), zb.tolist(), cc):
            M[rows[a], cols[b]] += c
        sv = np.linalg.svd(M, compute_uv=False)
        rank = int((sv > 1e-12 * sv[0]).sum())
        xa, xb = X & mask, X >> n_o
        if X == 0:
            kind = "diagonal"
        elif bin(X).count("1") == 2 and (xa == 0 or xb == 0):
            kind = "same-spin hop"
        else:
            kind = "other"
        out[(kind, rank)] += 1
    return out, len(xs)


@pytest.mark.parametrize("n_o,seed", [(3, 1), (4, 7), (6, 11)])
def test_phase_matrix_ranks(n_o, seed):
    ranks, n_groups = _group_ranks(n_o, seed)
    hops = 2 * comb(n_o, 2)
    assert ranks[("diagonal", n_o + 2)] == 1
    assert ranks[("same-spin hop", 2)] == hops
    assert ranks[("other", 1)] == n_groups - 1 - hops
    assert sum(ranks.values()) == n_groups
