"""Benchmark of the Pauli-sum operator-state path on one MI355X.

One step is one pass of the whole path on the 28-qubit molecular workload
(14 spatial orbitals, (7, 7) spin sector, D = 11,778,624): Jordan-Wigner
construction from device-resident integrals (string products + canonical
reduction), grouping by X-mask with the sector tables, the sector's rank
tables, the spin-factorized phase tables of the sector (group factors, beta
factors and move tables, alpha lists and images; --no-factor leaves them
out), H|psi> with complex64 storage and float64 accumulation, and the fused
float64 energy <psi|H|psi>.  The metric is amplitude*terms per second,
D * M / t_step with M the number of canonical Pauli strings.  Steps run
back to back as a serving loop runs them: each step's operator build (on a
second stream) overlaps the previous step's fused pass; the serial figure,
each build waiting for the previous pass, is reported beside it
(ms_per_step_serial).

The dominant kernel (the sector apply; for the Hubbard sector the rows
kernel) is timed with HIP events on the stream it runs on.  On the molecular
sector it is bound by vector-ALU issue:
its roofline is its VALU wave-instructions per launch (from the committed
rocprofv3 counters of the same kernel source) per second against 614.4 G/s,
with the measured HBM traffic and the method's algorithmic gather bytes,
D * b * (1 + G_conn) (b = 8 bytes per complex64 amplitude, G_conn connected
groups per target), reported beside it.  On the Hubbard sector it is bound by
HBM bandwidth and the algorithmic bytes are the roofline.  The complex128
(FP64 plain) apply is timed beside it, and the oracle's C twin is timed on a
bounded sample of the same workload on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4  # wave64 VALU issue: CUs x SIMDs x GHz / cycles per instruction
WORKLOADS = {
    # name: (kind, params); "bound" names the resource that limits the sector apply
    "molecular-28q-sector": ("molecular", dict(n_orb=14, n_alpha=7, n_beta=7, h_seed=2001, psi_seed=2101,
                                               bound="alu")),
    "molecular-12q-sector": ("molecular", dict(n_orb=6, n_alpha=3, n_beta=3, h_seed=1001, psi_seed=1102,
                                               bound="alu")),
    # the Hubbard sector's rows (103 KB) are too long to stage: with the
    # factor tables its apply is the rows kernel
    "hubbard-32q-sector": ("hubbard", dict(rows=4, cols=4, n_alpha=8, n_beta=8, psi_seed=4101, bound="hbm",
                                           kernel="rows")),
}


# sources that decide what the sector apply kernel does per launch: its
# device code, its launch planner and the tables grouping builds for it
APPLY_SOURCES = ("apply.hip", "factor.hip", "group.hip", "handles.h", "host_plan.h", "sector.h", "sector_c128_apply.hip",
                 "sector_c128_expval.hip", "sector_c64_apply.hip", "sector_c64_expval.hip")


def _source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2606_28952_amd", "csrc")
    for f in APPLY_SOURCES:
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            # code only: comment and blank-line edits do not change the kernels
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def _connected_groups(x_groups, n_orb, n_alpha, n_beta, weights=None):
    """Average number of groups whose source lies in the sector, per target:
    a group with masks (X_alpha, X_beta) connects a target iff each half flips
    as many occupied as empty orbitals; counted exactly by combinatorics.
    With ``weights`` (one per group, e.g. its number of strings) the average
    of the connected groups' weights summed per target."""
    from math import comb as _comb

    def comb(n, k):
        return _comb(n, k) if 0 <= k <= n else 0

    mask = (1 << n_orb) - 1
    total = 0
    da, db = comb(n_orb, n_alpha), comb(n_orb, n_beta)
    w = [1] * len(x_groups) if weights is None else [int(v) for v in weights]
    for x, wg in zip(x_groups.tolist(), w):
        xa, xb = x & mask, x >> n_orb
        pa, pb = bin(xa).count("1"), bin(xb).count("1")
        if pa % 2 or pb % 2:
            continue
        # targets whose alpha string has exactly pa/2 ones inside xa
        ca = comb(pa, pa // 2) * comb(n_orb - pa, n_alpha - pa // 2)
        cb = comb(pb, pb // 2) * comb(n_orb - pb, n_beta - pb // 2)
        total += ca * cb * wg
    return total / (da * db)


def _counters(kernel_tag):
    """Committed rocprofv3 counter summary of a kernel (HBM bytes and VALU
    wave-instructions per launch), or None when absent or taken on a
    different kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != _source_hash():
        return None
    return rec


def _host_cpu():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(h1, h2, n_orb, n_alpha, n_beta, psi, target_s=3.0):
    """The oracle's C twin (float64, term by term in scatter order, OpenMP)
    timed on a bounded sample of the same workload: every canonical string
    applied to all configurations of K whole source rows (alpha strings),
    scattered into the full output.  One warm-up, then the median of three
    runs, on all the threads OpenMP is given and on one thread; K is sized
    from the marginal cost of a row (two probes, so that the fixed cost of a
    call -- per-thread output partials and their sum -- does not count as
    row work) so that each run takes about target_s seconds."""
    from oracle import jw as ojw
    from oracle import native
    from oracle import space as ospace

    op = ojw.jw_sum(h1, h2)
    osp = ospace.SectorSpace(n_orb, n_alpha, n_beta)
    prep = native.prepare(op, osp)
    psi = np.asarray(psi, dtype=np.complex128)
    rows_all = np.linspace(0, osp.dim_alpha - 1, osp.dim_alpha, dtype=np.int64)
    rng = np.random.default_rng(0)

    def sources(k):
        rows = np.sort(rng.choice(rows_all, k, replace=False))
        return (rows[:, None] * osp.dim_beta + np.arange(osp.dim_beta)[None, :]).reshape(-1)

    def timed(k, threads):
        src = sources(k)
        t0 = time.perf_counter()
        _, used = native.apply_scatter(op, osp, psi, sources=src, threads=threads, prepared=prep)
        return time.perf_counter() - t0, used

    res = {}
    for name, threads in (("all", 0), ("one", 1)):
        timed(1, threads)                                # warm-up
        k1, k2 = (4, 16) if threads != 1 else (1, 2)
        d1, used = timed(k1, threads)
        d2, _ = timed(k2, threads)
        per_row = max((d2 - d1) / (k2 - k1), 1e-4)
        k = int(max(1, min(osp.dim_alpha, round(k1 + (target_s - d1) / per_row))))
        runs = sorted(timed(k, threads)[0] for _ in range(3))
        rate = k * osp.dim_beta * op.n_terms / runs[1]
        res[name] = (rate, used, k, runs[1])
    rate, used, k, t_med = res["all"]
    rate1, _, k1, t1 = res["one"]
    return {"value": rate, "unit": "amplitude*terms/s", "cores": used, "kind": "oracle",
            "sample": f"C/OpenMP float64 oracle, scatter order: all {op.n_terms} canonical strings applied to "
                      f"every configuration of {k} whole source rows ({k * osp.dim_beta} of {osp.dim} "
                      f"configurations), median of 3 runs ({t_med:.2f} s) on {used} threads",
            "value_1core": rate1,
            "sample_1core": f"{k1} source rows, median of 3 runs ({t1:.2f} s) on 1 thread",
            "full_apply_s_all_threads": osp.dim * op.n_terms / rate,
            "full_apply_s_1core": osp.dim * op.n_terms / rate1,
            "host": _host_cpu()}


def bench_batched(args):
    """Batched complex64 apply + energies in one launch vs per-job FP64 launches."""
    import torch

    import synth
    from paper_2606_28952_amd import api

    dev = torch.device("cuda:0")
    jobs32, jobs64, work = [], [], 0.0
    handles = []
    for n_orb, na, nb, hs, ps in synth.batched_sector_jobs():
        h1, h2 = synth.molecular_spin_integrals(n_orb, hs)
        H = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev))
        G = H.group()
        sp = api.Space.sector(n_orb, na, nb)
        if not args.no_factor:
            G.factor(sp)  # spin-factorized tables for the job's own sector
        psi = torch.from_numpy(synth.random_state(sp.dim, ps)).to(dev)
        p32 = psi.to(torch.complex64)
        jobs32.append((G, sp, p32, torch.empty_like(p32)))
        jobs64.append((G, sp, psi, torch.empty_like(psi)))
        handles.append(H)
        work += sp.dim * H.n_terms
    batch = api.Batch(jobs32)
    energies = torch.zeros(3 * len(jobs32), dtype=torch.float64, device=dev)

    def time_batch():
        for _ in range(args.warmup):
            batch.run(energies)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            batch.run(energies)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    t_default = time_batch()
    batch.set_config(128)  # persistent launch, default schedule otherwise
    t_persistent = time_batch()
    tuned_config, tuned_ms = batch.tune(reps=3)
    t_batch = time_batch()

    def time_graph(config):
        # the batch (under `config`) captured once in a HIP graph and replayed;
        # the replay must reproduce the eager outputs and energies exactly
        batch.set_config(config)
        batch.run(energies)
        torch.cuda.synchronize()
        eager = [torch.view_as_real(j[3]).clone() for j in jobs32] + [energies.clone()]
        graph, stream = torch.cuda.CUDAGraph(), torch.cuda.Stream()
        with torch.cuda.stream(stream):
            with torch.cuda.graph(graph, stream=stream):
                batch.run(energies)
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.replay()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        same = all(torch.equal(torch.view_as_real(j[3]), e) for j, e in zip(jobs32, eager)) and \
            torch.equal(energies, eager[-1])
        del graph
        return t, same

    t_graph, graph_same = time_graph(tuned_config)
    t_graph_persistent, graph_same_p = time_graph(128)
    batch.set_config(tuned_config)

    def per_job():
        for G, sp, psi, out in jobs64:
            api.apply_pauli_sum(G, sp, psi, out=out)

    def time_per_job():
        for _ in range(args.warmup):
            per_job()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            per_job()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    t_single = time_per_job()
    for G, _, _, _ in jobs64:
        G.set_factored(0)
    t_single_plain = time_per_job()
    for G, _, _, _ in jobs64:
        G.set_factored(0 if args.no_factor else 7)
    # accuracy of the batched complex64 results against FP64 on the same input
    worst = 0.0
    for (G, sp, p32, o32) in jobs32:
        ref = api.apply_pauli_sum(G, sp, p32.to(torch.complex128))
        worst = max(worst, (torch.linalg.vector_norm(o32.to(torch.complex128) - ref) /
                            torch.linalg.vector_norm(ref)).item())
    line = {
        "metric": "batched H|psi> amplitude*terms/s (64 jobs, complex64 storage, float64 accumulation)",
        "value": work / t_batch, "unit": "amplitude*terms/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_batch * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "complex64 storage, f64 accumulation", "data": "synthetic",
        "config": {"workload": "batched-64", "jobs": len(jobs32), "amplitude_terms": work,
                   "dims": [j[1].dim for j in jobs32], "factored": not args.no_factor},
        "ms_default_schedule": t_default * 1e3, "ms_persistent_schedule": t_persistent * 1e3,
        "tuned_schedule": tuned_config, "tuner_ms_per_run": tuned_ms, "work_items": batch.info()[2],
        "ms_graph_replay_tuned": t_graph * 1e3, "ms_graph_replay_persistent": t_graph_persistent * 1e3,
        "graph_replay_equals_eager": bool(graph_same and graph_same_p),
        "ms_per_job_fp64_launches": t_single * 1e3,
        "ms_per_job_fp64_launches_unfactored": t_single_plain * 1e3,
        "speedup_batched_c64_vs_per_job_fp64": t_single / t_batch,
        "speedup_batched_c64_vs_per_job_fp64_unfactored": t_single_plain / t_batch,
        "max_rel_err_c64_vs_fp64_same_input": worst,
    }
    print(json.dumps(line))


def bench_krylov(args):
    """4x4 periodic Hubbard (U = 4), (8, 8) sector: short-iterative Lanczos
    steps (12 vectors, dt = 0.05) from the Neel state, complex64 and complex128."""
    import torch

    import synth
    from paper_2606_28952_amd import api

    dev = torch.device("cuda:0")
    h1, h2 = synth.hubbard_spin_integrals(4, 4, t=1.0, u=4.0)
    G = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)).group()
    sp = api.Space.sector(16, 8, 8)
    if not args.no_factor:
        G.factor(sp)  # spin-factorized tables: the applies run the rows kernel
    na, nb = synth.neel_occupations(4, 4)
    start = sp.rank(torch.tensor([na | (nb << 16)], dtype=torch.int64, device=dev)).item()
    res = {}
    for name, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
        psi = torch.zeros(sp.dim, dtype=dtype, device=dev)
        psi[start] = 1.0
        prop = api.KrylovPropagator(G, sp, dtype=dtype, m=12)
        energies, norms = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.krylov_steps):
            info = prop.step(psi, 0.05)
            norms.append(info[0])
            energies.append(info[1])
            if (k + 1) % 25 == 0:
                print(f"[krylov {name}] {k + 1}/{args.krylov_steps} steps", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt_total = time.perf_counter() - t0
        res[name] = {"seconds": dt_total, "ms_per_step": dt_total * 1e3 / args.krylov_steps,
                     "norm_drift": max(abs(n - 1.0) for n in norms),
                     "energy_drift": max(energies) - min(energies), "energy0": energies[0], "psi": psi}
        del prop
    diff = (torch.linalg.vector_norm(res["c64"]["psi"].to(torch.complex128) - res["c128"]["psi"]) /
            torch.linalg.vector_norm(res["c128"]["psi"])).item()
    for r in res.values():
        r.pop("psi")
    print(json.dumps({"workload": "hubbard-32q-krylov", "steps": args.krylov_steps, "dt": 0.05, "vectors": 12,
                      "dim": sp.dim, "factored": not args.no_factor, "c64": res["c64"], "c128": res["c128"],
                      "final_state_rel_diff_c64_vs_c128": diff}))


def bench_pes(args):
    """Learned warm start on a potential-energy scan: 12 orbitals, (6, 6)
    reference, 24 qubits (full 2^24 space), 200 excitation rotations,
    R_j = j / (G - 1) for j < G geometries.  Every geometry runs the
    variational minimisation from the reference (cold) and from the network's
    prediction (warm, with the cold start as fallback); the network
    1 -> 256 -> 256 -> 200 is retrained on the converged parameters.  Prints
    one progress line per geometry on stderr and one JSON summary line."""
    import torch

    import synth
    from paper_2606_28952_amd import api, pes

    n_orb, na, nb, n_rot = 12, 6, 6, 200
    dev = torch.device("cuda:0")
    x, z = synth.excitation_masks(n_orb, na, nb, n_rot)
    ref = ((1 << na) - 1) | (((1 << nb) - 1) << n_orb)
    radii = np.linspace(0.0, 1.0, args.geometries)
    # cost of one energy + gradient evaluation at the middle of the scan
    h1, h2 = synth.pes_integrals(n_orb, 0.5)
    G = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)).group()
    _, n_groups, n_terms = G.info()
    # algorithmic gather bytes of one batched apply over all sector blocks:
    # sum over blocks of D_block * (1 + connected groups per target) amplitudes
    xg = G.read()[0]
    from math import comb

    gathers = sum(comb(n_orb, a) * comb(n_orb, b) * (1.0 + _connected_groups(xg, n_orb, a, b))
                  for a in range(n_orb + 1) for b in range(n_orb + 1))
    evals = {}
    for name, dtype in (("c128", torch.complex128), ("c64", torch.complex64)):
        v = api.VQE(G, n_orb, x, z, ref, dtype=dtype)
        th = np.random.default_rng(0).normal(size=n_rot) * 0.05
        v.energy_grad(th)
        t0 = time.perf_counter()
        for _ in range(3):
            v.energy_grad(th)
        t_eg = (time.perf_counter() - t0) / 3
        t0 = time.perf_counter()
        for _ in range(3):
            v.energy(th)
        evals[name] = {"energy_grad_ms": t_eg * 1e3, "energy_ms": (time.perf_counter() - t0) / 3 * 1e3}
        del v
    del G

    def log(j, r):
        print(f"[pes] {j + 1}/{len(radii)} R={r['R']:.4f} cold {r['E_cold']:.10f} ({r['iters_cold']} it) "
              f"warm[{r['start']}] {r['E_warm']:.10f} ({r['iters_warm']} it) {r['sec_total']:.1f}s",
              file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    recs = pes.scan(lambda r: synth.pes_integrals(n_orb, r), radii, n_orb, x, z, ref, dtype=torch.complex128,
                    hidden=256, mlp_params=synth.mlp_init(256, n_rot, seed=2), train_steps=600, lr=1e-3,
                    g_tol=1e-5, log=log)
    wall = time.perf_counter() - t0
    summ = pes.summary(recs)
    out = {"workload": "pes-scan-24q", "n_qubits": 2 * n_orb, "dim": 1 << (2 * n_orb), "rotations": n_rot,
           "geometries": len(radii), "pauli_strings_R0.5": n_terms, "groups_R0.5": n_groups,
           "apply_gather_amplitudes_R0.5": gathers,
           "integrals": {"form": "h(R) = h0 + s (R h1 + R^2 h2), g(R) likewise", "s": 0.3, "basis": "eigenbasis of h0",
                         "seeds": [5001, 5002, 5003],
                         "change": "differs from plain h0 + R h1 + R^2 h2 in the draws' own basis: the R terms "
                                   "are scaled by s = 0.3 and every term is expressed in h0's eigenbasis, so the "
                                   "(6, 6) reference is h0's one-body ground state (as Hartree-Fock orbitals make "
                                   "it) and the scan starts near a mean-field solution"},
           "network": "1-256-256-200 bf16/fp32", "dtype": "c128 (fp64 energies)",
           "g_tol": 1e-5, "wall_s": wall, "evaluation": evals, **summ,
           "sec_cold": sum(r["sec_cold"] for r in recs), "sec_warm": sum(r["sec_warm"] for r in recs),
           "sec_train": sum(r.get("sec_train", 0.0) for r in recs),
           "per_geometry": [{k: r[k] for k in ("R", "E_ref", "E_cold", "iters_cold", "E_warm", "iters_warm",
                                                "start")} for r in recs]}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="molecular-28q-sector",
                    choices=sorted(WORKLOADS) + ["batched-64", "hubbard-krylov", "pes-scan"])
    ap.add_argument("--geometries", type=int, default=40, help="pes-scan: number of geometries")
    ap.add_argument("--krylov-steps", type=int, default=200)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="counter calibration: one device-to-device copy of this many bytes, nothing else")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-factor", action="store_true",
                    help="skip the spin-factorized phase tables (unfactored evaluation throughout)")
    ap.add_argument("--apply-only", type=int, default=0,
                    help="profiling mode: run only N sector applies (complex64) after setup, print nothing else")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); this path has no multi-GPU mode.",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_bytes:
        import torch

        src = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copied {src.numel() * 4} bytes")
        return
    if args.workload == "batched-64":
        return bench_batched(args)
    if args.workload == "hubbard-krylov":
        return bench_krylov(args)
    if args.workload == "pes-scan":
        return bench_pes(args)

    import torch

    import synth
    from paper_2606_28952_amd import api

    kind, prm = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if kind == "molecular":
        n_orb = prm["n_orb"]
        h1, h2 = synth.molecular_spin_integrals(n_orb, prm["h_seed"])
    else:
        n_orb = prm["rows"] * prm["cols"]
        h1, h2 = synth.hubbard_spin_integrals(prm["rows"], prm["cols"])
    na, nb = prm["n_alpha"], prm["n_beta"]
    h1_d = torch.from_numpy(h1).to(dev)
    h2_d = torch.from_numpy(h2).to(dev)
    psi64_np = synth.random_state(_dim(n_orb, na, nb), prm["psi_seed"])
    psi32 = torch.from_numpy(psi64_np.astype(np.complex64)).to(dev)
    out32 = torch.empty_like(psi32)
    res = torch.empty(3, dtype=torch.float64, device=dev)

    def build():
        H = api.jw_transform(h1_d, h2_d)
        G = H.group()
        sp = api.Space.sector(n_orb, na, nb)
        if not args.no_factor:
            G.factor(sp)  # spin-factorized phase tables for this beta sector
        return H, G, sp

    if args.apply_only:
        _, G, sp = build()
        work0 = torch.empty(max(1, sp.workspace_bytes() // 8), dtype=torch.float64, device=dev)
        for _ in range(args.apply_only):
            api.expval(G, sp, psi32, work=work0, result=res, out=out32)
        torch.cuda.synchronize()
        print(f"apply-only done: {args.apply_only} launches")
        return

    H, G, sp = build()
    work = torch.empty(max(1, sp.workspace_bytes() // 8), dtype=torch.float64, device=dev)
    D = sp.dim
    M = H.n_terms
    xg, goff = G.read()[:2]
    g_conn = _connected_groups(xg, n_orb, na, nb)
    t_conn = _connected_groups(xg, n_orb, na, nb, weights=np.diff(goff.astype(np.int64)))
    del H, G, sp

    # Steps run back to back as a serving loop runs them: step k + 1's
    # operator build (host work and small kernels, on a second stream)
    # overlaps step k's fused pass on the first.  Every step builds its own
    # operator and applies it.  The handles of finished steps are destroyed
    # after the timed region: destroying one frees device memory, which
    # waits for the whole device.  `pipelined=False` waits for each fused
    # pass before the next build (the serial figure reported beside it).
    main_s, side_s = torch.cuda.Stream(), torch.cuda.Stream()  # default priority

    def run_steps(n, evs=None, pipelined=True):
        keep = []

        def build_async():
            with torch.cuda.stream(side_s):
                hgs = build()
                ready = torch.cuda.Event()
                ready.record(side_s)
            keep.append(hgs)
            return hgs, ready

        nxt = build_async()
        for k in range(n):
            (_, G, sp), ready = nxt
            main_s.wait_event(ready)
            with torch.cuda.stream(main_s):
                # H|psi> and <psi|H|psi> come from one fused pass of the sector kernel
                if evs:
                    evs[k][0].record(main_s)
                api.expval(G, sp, psi32, work=work, result=res, out=out32)
                if evs:
                    evs[k][1].record(main_s)
            if k + 1 < n:
                if not pipelined:
                    main_s.synchronize()
                nxt = build_async()
        torch.cuda.synchronize()
        return keep

    def timed(pipelined):
        keep = run_steps(args.warmup, pipelined=pipelined)
        del keep
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        keep = run_steps(args.steps, evs, pipelined)
        t1 = time.perf_counter()
        del keep
        return (t1 - t0) * 1e3 / args.steps, float(np.mean([a.elapsed_time(b) for a, b in evs]))

    ms_step_serial, apply_ms_serial = timed(False)
    energy_serial = res.cpu().numpy()
    ms_step, apply_ms = timed(True)
    energy = res.cpu().numpy()
    # every step builds and applies the same operator to the same state, and
    # the kernels are deterministic: both loops must end on the same bits
    pipelined_equals_serial = bool(np.array_equal(energy, energy_serial))

    # FP64 plain (complex128 storage) vs complex64 storage, apply kernel only
    _, G, sp = build()
    psi64 = torch.from_numpy(psi64_np).to(dev)
    out64 = torch.empty_like(psi64)

    def time_apply(psi, out, reps=10):
        api.apply_pauli_sum(G, sp, psi, out=out)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            api.apply_pauli_sum(G, sp, psi, out=out)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    c64_ms = time_apply(psi32, out32)
    c128_ms = time_apply(psi64, out64)

    # one device's share of an eight-way split of the target alpha rows
    # (the row-range entry point; each share needs the whole state): the
    # kernel time of each share at its real shape, complex64
    def time_share(a0, a1, reps=10):
        o = out32[a0 * sp.shape()[4]:a1 * sp.shape()[4]]
        api.apply_pauli_sum_rows(G, sp, psi32, a0, a1, out=o)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            api.apply_pauli_sum_rows(G, sp, psi32, a0, a1, out=o)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    dim_alpha = sp.shape()[3]
    share_ms = [time_share(r * dim_alpha // 8, (r + 1) * dim_alpha // 8) for r in range(8)]
    # the unfactored evaluation of the same kernel, for comparison
    G.set_factored(0)
    c64_plain_ms = time_apply(psi32, torch.empty_like(psi32))
    c128_plain_ms = time_apply(psi64, torch.empty_like(psi64))
    G.set_factored(0 if args.no_factor else 7)
    # storage error of the complex64 path: against complex128 on the same
    # FP32-rounded input (kernel error) and against the FP64 state
    ref_same = api.apply_pauli_sum(G, sp, psi32.to(torch.complex128))
    err_kernel = (torch.linalg.vector_norm(out32.to(torch.complex128) - ref_same) /
                  torch.linalg.vector_norm(ref_same)).item()
    err_state = (torch.linalg.vector_norm(out32.to(torch.complex128) - out64) /
                 torch.linalg.vector_norm(out64)).item()
    e64 = api.expval(G, sp, psi64).cpu().numpy()
    e32 = api.expval(G, sp, psi32).cpu().numpy()

    # roofline of the dominant kernel.  The sector apply is bound by vector-ALU
    # issue (one wave64 VALU instruction per 4 cycles per SIMD: 256 CUs x 4
    # SIMDs x 2.4 GHz / 4 = 614.4 G wave-instructions/s); its VALU count and
    # HBM bytes per launch come from the committed counter runs of the same
    # kernel source (null when the kernel has changed since).  The method's
    # algorithmic gather bytes per launch, D * 8 B * (1 + G_conn), are
    # reported beside it: most of them are served from LDS and caches.
    # HBM bandwidth a plain device-to-device copy reaches on this device
    # (1 GiB read + 1 GiB written), reported beside the published peak
    cp_src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    cp_dst = torch.empty_like(cp_src)
    cp_dst.copy_(cp_src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        cp_dst.copy_(cp_src)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * cp_src.numel() * 4 * 5 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del cp_src, cp_dst
    bytes_per_launch = D * 8 * (1.0 + g_conn)
    gather_gbs = bytes_per_launch / (apply_ms * 1e-3) / 1e9
    kernel_tag = f"apply_{prm.get('kernel', 'sector') if not args.no_factor else 'sector'}_c64_{args.workload}"
    ctr = _counters(kernel_tag)
    traffic = ctr.get("hbm_bytes_per_launch") if ctr else None
    valu = ctr.get("valu_wave_insts_per_launch") if ctr else None
    valu_peak = VALU_PEAK_GINST
    if prm["bound"] == "hbm":
        # bandwidth-bound (few groups per target, rows too long for LDS): the
        # algorithmic gather bytes against the HBM peak
        roofline = {"bound": "hbm", "achieved": gather_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": gather_gbs / HBM_PEAK_GBS, "measured_copy_GBs": copy_gbs, "traffic": traffic,
                    "hbm_GBs": traffic / (apply_ms * 1e-3) / 1e9 if traffic else None,
                    "valu_frac": valu / (apply_ms * 1e-3) / 1e9 / valu_peak if valu else None,
                    "apply_ms": apply_ms, "apply_ms_serial_steps": apply_ms_serial}
    else:
        roofline = {"bound": "alu", "resource": "VALU issue (wave64 instructions)",
                    "achieved": valu / (apply_ms * 1e-3) / 1e9 if valu else None, "peak": valu_peak,
                    "unit": "G VALU wave-instructions/s",
                    "frac": valu / (apply_ms * 1e-3) / 1e9 / valu_peak if valu else None,
                    "traffic": traffic,
                    "hbm_GBs": traffic / (apply_ms * 1e-3) / 1e9 if traffic else None,
                    "hbm_frac": traffic / (apply_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if traffic else None,
                    "measured_copy_GBs": copy_gbs,
                    "algorithmic_gather_bytes": bytes_per_launch, "algorithmic_gather_GBs": gather_gbs,
                    "apply_ms": apply_ms, "apply_ms_serial_steps": apply_ms_serial}
    line = {
        "metric": "H|psi> amplitude*terms/s (complex64 storage, float64 accumulation)",
        "value": D * M / (ms_step * 1e-3),
        "unit": "amplitude*terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_serial": ms_step_serial,
        "pipelined_equals_serial": pipelined_equals_serial,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "complex64 storage, f64 accumulation",
        "data": "synthetic (seeded Gaussian integrals and states)",
        "config": {"workload": args.workload, "n_orb": n_orb, "n_alpha": na, "n_beta": nb, "dim": D,
                   "n_strings": M, "groups_connected_per_target": round(g_conn, 3),
                   "strings_connected_per_target": round(t_conn, 3), "storage": "complex64",
                   "step": "jw_transform+group_by_xmask+space_sector+" +
                           ("" if args.no_factor else "grouped_factor+") + "fused(apply_pauli_sum+expval)"},
        "roofline": roofline,
        "apply_ms_c64": c64_ms,
        "apply_ms_c128": c128_ms,
        "apply_rate_c64": D * M / (c64_ms * 1e-3),
        "apply_connected_rate_c64": D * t_conn / (c64_ms * 1e-3),
        "apply_rate_c128": D * M / (c128_ms * 1e-3),
        "speedup_c64_vs_c128": c128_ms / c64_ms,
        "factored": not args.no_factor,
        "apply_ms_c64_row_shares_of_8": [round(t, 4) for t in share_ms],
        "apply_ms_c64_unfactored": c64_plain_ms,
        "apply_ms_c128_unfactored": c128_plain_ms,
        "rel_err_c64_vs_c128_same_input": err_kernel,
        "rel_err_c64_vs_fp64_state": err_state,
        "energy_c64": float(e32[0]),
        "energy_c128": float(e64[0]),
        "energy_diff_c64_c128": float(e32[0] - e64[0]),
        "energy_step": float(energy[0]),
        "kernel_source": _source_hash(),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(h1, h2, n_orb, na, nb, psi64_np)
    print(json.dumps(line))


def _dim(n_orb, na, nb):
    from math import comb

    return comb(n_orb, na) * comb(n_orb, nb)


if __name__ == "__main__":
    main()
