"""pbs_expval_noalloc (fixed library workspace, no allocation) against
pbs_expval (caller workspace): the same kernels and reduction order, so the
energy triple and the stored H psi must be bit-identical.  Two calls in a
row, the second on a smaller space, show that nothing of the first call's
workspace contents leaks into the second; a space whose partials exceed the
fixed workspace is refused before anything runs."""

from ctypes import c_void_p

import numpy as np
import pytest
import torch

import synth
from paper_2606_28952_amd import _abi, api


def _case(dev, n_orb, na, nb, seed, dtype):
    h1, h2 = synth.molecular_spin_integrals(n_orb, seed)
    H = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev))
    G = H.group()
    sp = api.Space.sector(n_orb, na, nb)
    psi = torch.from_numpy(synth.random_state(sp.dim, seed + 100)).to(dev).to(dtype)
    return G, sp, psi


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_noalloc_matches_expval_twice_shrinking(dev, dtype):
    # larger sector first (n_o = 10, D = 63,504), then a smaller one (n_o = 6, D = 400)
    for n_orb, na, nb, seed in [(10, 5, 5, 31), (6, 3, 3, 37)]:
        G, sp, psi = _case(dev, n_orb, na, nb, seed, dtype)
        out_ref = torch.empty_like(psi)
        res_ref = api.expval(G, sp, psi, out=out_ref)
        out_na = torch.full_like(psi, float("nan"))
        res_na = torch.full((3,), float("nan"), dtype=torch.float64, device=dev)
        api.expval_noalloc(G, sp, psi, res_na, out=out_na)
        torch.cuda.synchronize()
        a, b = res_ref.cpu().numpy(), res_na.cpu().numpy()
        assert a.tobytes() == b.tobytes(), (n_orb, a, b)
        assert torch.equal(torch.view_as_real(out_ref), torch.view_as_real(out_na)), n_orb
        # and without storing H psi
        res2 = torch.full((3,), float("nan"), dtype=torch.float64, device=dev)
        api.expval_noalloc(G, sp, psi, res2)
        assert res2.cpu().numpy().tobytes() == a.tobytes(), n_orb
        # the energy itself, against the dot product of the stored H psi
        e = np.vdot(psi.cpu().numpy().astype(np.complex128), out_ref.cpu().numpy().astype(np.complex128))
        tol = 1e-12 if dtype == torch.complex128 else 1e-6
        assert abs(a[0] - e.real) <= tol * max(1.0, abs(e)), (a[0], e)


@pytest.mark.gpu
def test_noalloc_full_space(dev):
    h1, h2 = synth.molecular_spin_integrals(4, 5)
    G = api.jw_transform(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)).group()
    sp = api.Space.full(8)
    psi = torch.from_numpy(synth.random_state(sp.dim, 6)).to(dev)
    res_ref = api.expval(G, sp, psi)
    res_na = torch.empty(3, dtype=torch.float64, device=dev)
    api.expval_noalloc(G, sp, psi, res_na)
    assert res_ref.cpu().numpy().tobytes() == res_na.cpu().numpy().tobytes()


@pytest.mark.gpu
def test_noalloc_refuses_spaces_beyond_its_workspace(dev):
    # 36 qubits, (9, 9) sector: 48,620 rows of 48,620 columns need far more
    # partials than the fixed workspace holds; refused before any launch
    x = np.zeros(1, np.uint64)
    z = np.ones(1, np.uint64)
    G = api.PauliSum.create(36, x, z, np.ones(1, np.complex128)).canonicalize().group()
    sp = api.Space.sector(18, 9, 9)
    need = sp.workspace_bytes()
    lib = _abi.lib()
    assert need > lib_max_bytes()
    dummy = torch.zeros(4, dtype=torch.complex64, device=dev)
    res = torch.zeros(3, dtype=torch.float64, device=dev)
    st = lib.pbs_expval_noalloc(G._h, sp._h, api.PBS_C64, c_void_p(dummy.data_ptr()), None,
                                c_void_p(res.data_ptr()), None)
    msg = lib.pbs_last_error().decode(errors="replace")
    assert st == 2, msg
    assert "fixed workspace" in msg
    torch.cuda.synchronize()
    assert torch.count_nonzero(res).item() == 0


def lib_max_bytes():
    import os
    import re

    hdr = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "pbs.h")
    m = re.search(r"#define PBS_EXPVAL_NOALLOC_MAX_BYTES \((\d+)u \* 1024u \* 1024u\)", open(hdr).read())
    return int(m.group(1)) << 20
