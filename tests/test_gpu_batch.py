"""GPU tests of the batched launch (pbs_batch_*): parity with single launches
and with the oracle, fused energies, and replay inside a captured HIP graph."""

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


# (n_orb, N_alpha, N_beta, integral seed, state seed): uneven sectors, own operators
JOBS = [(4, 2, 2, 11, 21), (5, 2, 3, 12, 22), (6, 3, 3, 13, 23), (7, 3, 2, 14, 24), (6, 1, 4, 15, 25),
        (7, 4, 3, 16, 26), (3, 1, 1, 17, 27), (8, 4, 4, 18, 28)]


def _build(dev, dtype, factor=False):
    api = _api()
    jobs, refs = [], []
    for n_o, na, nb, hs, ps in JOBS:
        h1, h2 = synth.molecular_spin_integrals(n_o, hs)
        G = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)).group()
        sp = api.Space.sector(n_o, na, nb)
        if factor:
            G.factor(sp)  # spin-factorized tables for this job's beta sector
        psi_np = synth.random_state(sp.dim, ps)
        if dtype == torch.complex64:
            psi_np = psi_np.astype(np.complex64).astype(np.complex128)
        psi = torch.from_numpy(psi_np).to(dev).to(dtype)
        out = torch.empty_like(psi)
        jobs.append((G, sp, psi, out))
        refs.append((h1, h2, n_o, na, nb, psi_np))
    return jobs, refs


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_batch_matches_single_launches_and_oracle(dev, dtype):
    api = _api()
    jobs, refs = _build(dev, dtype)
    batch = api.Batch(jobs)
    energies = torch.zeros(3 * len(jobs), dtype=torch.float64, device=dev)
    batch.run()
    torch.cuda.synchronize()
    outs = [j[3].clone() for j in jobs]
    batch.run(energies)
    torch.cuda.synchronize()
    e = energies.cpu().numpy().reshape(-1, 3)
    for k, ((G, sp, psi, out), (h1, h2, n_o, na, nb, psi_np)) in enumerate(zip(jobs, refs)):
        single = api.apply_pauli_sum(G, sp, psi)
        assert torch.equal(torch.view_as_real(single), torch.view_as_real(outs[k])), f"job {k} differs from single"
        assert torch.equal(torch.view_as_real(out), torch.view_as_real(outs[k])), f"job {k} differs between runs"
        ref = oapply.apply_scatter(ojw.jw_sum(h1, h2), ospace.SectorSpace(n_o, na, nb), psi_np)
        tol = 1e-12 if dtype == torch.complex128 else 1e-6
        assert rel_err(out.cpu().numpy(), ref) < tol
        e_ref = np.vdot(psi_np, ref)
        assert abs(e[k, 0] - e_ref.real) < 1e-11 * max(1.0, abs(e_ref))
        assert abs(e[k, 2] - np.vdot(psi_np, psi_np).real) < 1e-12
        ev_single = api.expval(G, sp, psi).cpu().numpy()
        assert abs(ev_single[0] - e[k, 0]) < 1e-12 * max(1.0, abs(e_ref))


@pytest.mark.parametrize("config", [0, 128], ids=["grid", "persistent"])
def test_batch_graph_replay(dev, config):
    api = _api()
    jobs, _ = _build(dev, torch.complex64)
    batch = api.Batch(jobs)
    batch.set_config(config)
    energies = torch.zeros(3 * len(jobs), dtype=torch.float64, device=dev)
    batch.run(energies)
    torch.cuda.synchronize()
    eager_out = [j[3].clone() for j in jobs]
    eager_e = energies.clone()
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    for j in jobs:
        j[3].zero_()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            batch.run(energies)
    torch.cuda.synchronize()
    for rep in range(3):
        for j in jobs:
            j[3].zero_()          # eager work between replays
        energies.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k, j in enumerate(jobs):
            assert torch.equal(torch.view_as_real(j[3]), torch.view_as_real(eager_out[k])), f"replay {rep} job {k}"
        assert torch.equal(energies, eager_e), f"replay {rep} energies"


def test_batch_rejects_bad_jobs(dev):
    api = _api()
    from paper_2606_28952_amd._abi import PbsError

    jobs, _ = _build(dev, torch.complex128)
    G, sp, psi, out = jobs[0]
    with pytest.raises(PbsError, match="overlaps"):
        api.Batch([(G, sp, psi, psi)])
    with pytest.raises(PbsError, match="outputs of jobs overlap"):
        api.Batch([(G, sp, psi, out), (G, sp, psi.clone(), out)])
    with pytest.raises(PbsError, match="spin-sector"):
        h1, h2 = synth.molecular_spin_integrals(3, 1)
        Gf = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)).group()
        x = torch.zeros(64, dtype=torch.complex128, device=dev)
        api.Batch([(Gf, api.Space.full(6), x, torch.zeros_like(x))])
    with pytest.raises(TypeError):
        api.Batch([(G, sp, psi, out), (G, sp, psi.to(torch.complex64), out.to(torch.complex64))])


def _oracle_refs(refs):
    out = []
    for h1, h2, n_o, na, nb, psi_np in refs:
        ref = oapply.apply_scatter(ojw.jw_sum(h1, h2), ospace.SectorSpace(n_o, na, nb), psi_np)
        out.append((ref, np.vdot(psi_np, ref).real))
    return out


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_every_schedule_matches_oracle(dev, dtype):
    api = _api()
    jobs, refs = _build(dev, dtype, factor=True)
    want = _oracle_refs(refs)
    batch = api.Batch(jobs)
    tol = 1e-12 if dtype == torch.complex128 else 1e-6
    energies = torch.zeros(3 * len(jobs), dtype=torch.float64, device=dev)
    first = {}  # flags -> outputs under the first workgroup order tried
    for config in range(256):
        batch.set_config(config)
        assert batch.info()[0] == config and batch.info()[1] == -1.0
        for _, _, _, out in jobs:
            out.zero_()
        batch.run(energies)
        torch.cuda.synchronize()
        e = energies.cpu().numpy().reshape(-1, 3)
        for k, ((_, _, _, out), (ref, e_ref)) in enumerate(zip(jobs, want)):
            assert rel_err(out.cpu().numpy(), ref) < tol, (config, k)
            assert abs(e[k, 0] - e_ref) < 1e-11 * max(1.0, abs(e_ref)), (config, k)
        # the workgroup order moves work between workgroups, never within a target
        outs = [torch.view_as_real(j[3]).clone() for j in jobs]
        # a persistent launch (128) moves items between workgroups too
        flags = config & (15 | 64)
        if flags in first:
            assert all(torch.equal(a, b) for a, b in zip(outs, first[flags])), config
        else:
            first[flags] = outs


def test_tuner_keeps_the_fastest_schedule(dev):
    api = _api()
    jobs, refs = _build(dev, torch.complex64)
    want = _oracle_refs(refs)
    batch = api.Batch(jobs)
    wg0 = batch.info()[2]
    config, ms = batch.tune(reps=2)
    assert 0 <= config < 256 and ms > 0.0
    assert batch.info() == (config, ms, wg0)  # the workgroup count does not depend on the schedule
    for _, _, _, out in jobs:
        out.zero_()
    batch.run()
    torch.cuda.synchronize()
    for (_, _, _, out), (ref, _) in zip(jobs, want):
        assert rel_err(out.cpu().numpy(), ref) < 1e-6
    with pytest.raises(Exception, match="schedule"):
        batch.set_config(256)


def test_config3_batch_of_64_uneven_sectors(dev):
    """The 64-job batch at its full sizes (n_orb 10 to 13, 20 to 26 qubits,
    D from 30,240 to 2,944,656, each job its own operator), complex64
    storage, in one launch with energies: unfactored with the default
    schedule, then with the spin-factorized tables of every job in a
    persistent launch (the configuration the benchmark times).  Every job
    equals its single launch bit for bit; six 13-orbital jobs (every electron
    count and both S_z values among them) are checked on 8 whole rows against
    the oracle's C twin, and four 10-orbital jobs on the whole vector and the
    energy."""
    from oracle import native

    api = _api()
    specs = synth.batched_sector_jobs()
    jobs, inputs = [], []
    for n_o, na, nb, hs, ps in specs:
        h1, h2 = synth.molecular_spin_integrals(n_o, hs)
        G = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)).group()
        sp = api.Space.sector(n_o, na, nb)
        psi32 = synth.random_state(sp.dim, ps).astype(np.complex64)
        t = torch.from_numpy(psi32).to(dev)
        jobs.append((G, sp, t, torch.empty_like(t)))
        inputs.append((h1, h2, psi32))
    print(f"[batch64] {len(jobs)} jobs, {sum(j[1].dim for j in jobs)} amplitudes", flush=True)
    row_refs, vec_refs = {}, {}
    for k in (3, 7, 11, 15, 19, 63):          # n_orb = 13
        n_o, na, nb, _, _ = specs[k]
        h1, h2, psi32 = inputs[k]
        osp = ospace.SectorSpace(n_o, na, nb)
        rows = np.random.default_rng(k).choice(osp.dim_alpha, 8, replace=False)
        tgt = (rows[:, None] * osp.dim_beta + np.arange(osp.dim_beta)[None, :]).reshape(-1)
        row_refs[k] = (torch.from_numpy(tgt).to(dev), native.apply_targets(ojw.jw_sum(h1, h2), osp, psi32, tgt)[0])
    for k in (0, 20, 40, 60):                 # n_orb = 10
        n_o, na, nb, _, _ = specs[k]
        h1, h2, psi32 = inputs[k]
        ref, _ = native.apply_scatter(ojw.jw_sum(h1, h2), ospace.SectorSpace(n_o, na, nb), psi32)
        vec_refs[k] = (ref, np.vdot(psi32.astype(np.complex128), ref).real)

    def check(batch, label):
        energies = torch.zeros(3 * len(jobs), dtype=torch.float64, device=dev)
        for _, _, _, out in jobs:
            out.zero_()
        batch.run(energies)
        torch.cuda.synchronize()
        e = energies.cpu().numpy().reshape(-1, 3)
        for k, (G, sp, t, out) in enumerate(jobs):
            single = api.apply_pauli_sum(G, sp, t)
            assert torch.equal(torch.view_as_real(single), torch.view_as_real(out)), f"{label} job {k}"
        for k, (tsel, ref) in row_refs.items():
            got = jobs[k][3][tsel].cpu().numpy().astype(np.complex128)
            assert rel_err(got, ref) < 1e-6, f"{label} job {k}"
        for k, (ref, e_ref) in vec_refs.items():
            assert rel_err(jobs[k][3].cpu().numpy().astype(np.complex128), ref) < 1e-6, f"{label} job {k}"
            assert abs(e[k, 0] - e_ref) < 1e-8, f"{label} job {k}"

    check(api.Batch(jobs), "unfactored")
    print("[batch64] factored, persistent", flush=True)
    for G, sp, _, _ in jobs:
        G.factor(sp)
    batch = api.Batch(jobs)
    batch.set_config(128)  # PBS_BATCH_PERSISTENT
    check(batch, "factored persistent")
