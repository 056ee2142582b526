"""Potential-energy scan with a learned warm start for the variational step.

Along a scan R_0 < R_1 < ... each geometry's Hamiltonian H(R) is built from
its integrals by the library's Jordan-Wigner construction and grouped; the
Pauli-rotation ansatz energy E(theta) = <psi(theta)|H(R)|psi(theta)>
(Section 2.1, Eq. vqe_energy) is minimised by L-BFGS (Section 3.2 uses the
same optimiser, from scratch at every geometry).  The warm start adds a
network theta(R) trained on the parameters converged at the earlier
geometries: its prediction is the starting point, and the cold start
theta = 0 (the reference state) is the fallback whenever the network is
untrained or its prediction has a higher energy than the reference.

Every numerical step runs in the HIP library (construction, grouping,
energies and gradients, network training and inference); this module only
sequences the calls and records what happened.
"""

import time

import numpy as np
import torch

from . import api


def scan(integrals, radii, n_orb, gen_x, gen_z, ref, *, dtype=torch.complex128, hidden=256, mlp_params=None,
         train_steps=600, lr=1e-3, min_train=1, max_iter=500, g_tol=1e-5, f_tol=0.0, run_cold=True, log=None):
    """Runs the scan.

    integrals(R) -> (h1, h2) spin-orbital arrays (float64, host);
    gen_x, gen_z: uint64 X and Z masks of the Hermitian rotation generators
    P_k (bit q = qubit q, phase 0, applied in order), as ``api.VQE`` takes
    them;
    ref: reference basis state; mlp_params: packed float32 initial network
    parameters (``api.MLP`` layout) for hidden width ``hidden``.
    Returns a list of per-geometry records (dicts)."""
    dev = torch.device("cuda")
    x = np.ascontiguousarray(gen_x, dtype=np.uint64)
    z = np.ascontiguousarray(gen_z, dtype=np.uint64)
    if x.shape != z.shape or x.ndim != 1:
        raise ValueError("gen_x and gen_z must be 1-D arrays of one mask per rotation")
    n_rot = len(x)
    net = api.MLP(hidden, n_rot, max(1, len(radii)), mlp_params) if mlp_params is not None else None
    seen_r, seen_theta = [], []
    records = []
    for j, r in enumerate(radii):
        t0 = time.perf_counter()
        h1, h2 = integrals(r)
        G = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)).group()
        vqe = api.VQE(G, n_orb, x, z, ref, dtype=dtype)
        zero = np.zeros(n_rot)
        e_ref = vqe.energy(zero)
        rec = {"R": float(r), "E_ref": e_ref}
        if run_cold:
            t = time.perf_counter()
            th_c, e_c, it_c, ev_c, why_c = vqe.minimize(zero, max_iter=max_iter, g_tol=g_tol, f_tol=f_tol)
            rec.update(E_cold=e_c, iters_cold=it_c, evals_cold=ev_c, stop_cold=why_c,
                       sec_cold=time.perf_counter() - t)
        if net is not None:
            t = time.perf_counter()
            start, source, e_start, probe = zero, "cold", e_ref, 0
            if len(seen_r) >= min_train:
                probe = 1  # the energy of the prediction is one more evaluation
                guess = net.forward(torch.tensor([r], dtype=torch.float32, device=dev)).cpu().numpy()[0]
                guess = guess.astype(np.float64)
                e_guess = vqe.energy(guess)
                if e_guess < e_ref:
                    start, source, e_start = guess, "network", e_guess
            th_w, e_w, it_w, ev_w, why_w = vqe.minimize(start, max_iter=max_iter, g_tol=g_tol, f_tol=f_tol)
            rec.update(E_warm=e_w, iters_warm=it_w, evals_warm=ev_w + probe, stop_warm=why_w, start=source,
                       E_start=e_start, sec_warm=time.perf_counter() - t)
            seen_r.append(r)
            seen_theta.append(th_w)
            if train_steps > 0:
                t = time.perf_counter()
                xs = torch.tensor(seen_r, dtype=torch.float32, device=dev)
                ts = torch.tensor(np.array(seen_theta), dtype=torch.float32, device=dev)
                losses = net.train(xs, ts, train_steps, lr)
                rec.update(train_loss=float(losses[-1].item()), sec_train=time.perf_counter() - t)
        rec["sec_total"] = time.perf_counter() - t0
        records.append(rec)
        if log is not None:
            log(j, rec)
        del vqe, G
    return records


def summary(records):
    """Totals of a scan: iterations and evaluations of the cold and warm
    paths, and the largest energy gap between them."""
    out = {"geometries": len(records)}
    if records and "iters_cold" in records[0]:
        out["iters_cold"] = int(sum(r["iters_cold"] for r in records))
        out["evals_cold"] = int(sum(r["evals_cold"] for r in records))
    if records and "iters_warm" in records[0]:
        out["iters_warm"] = int(sum(r["iters_warm"] for r in records))
        out["evals_warm"] = int(sum(r["evals_warm"] for r in records))
        out["network_starts"] = int(sum(r["start"] == "network" for r in records))
    if "iters_cold" in out and "iters_warm" in out:
        gaps = [r["E_warm"] - r["E_cold"] for r in records]
        out["max_E_warm_minus_cold"] = float(max(gaps))
        out["min_E_warm_minus_cold"] = float(min(gaps))
    return out
