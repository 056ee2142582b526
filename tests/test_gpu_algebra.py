"""GPU parity of the Pauli algebra through the C ABI, bit-exact against the
oracle: string products, canonical reduction, sum products and the
Jordan-Wigner Hamiltonian."""

import numpy as np
import pytest
import torch

import synth
from oracle import jw as ojw
from oracle import pauli as opauli
from oracle.pauli import PauliSum as OSum

pytestmark = pytest.mark.gpu


def _api():
    from paper_2606_28952_amd import api

    return api


def _oracle_mul(n, xa, za, pa, xb, zb, pb):
    la = opauli.xz_to_letters(xa, za, n)
    lb = opauli.xz_to_letters(xb, zb, n)
    lo, po = opauli.string_product(la, pa, lb, pb)
    xo, zo = opauli.letters_to_xz(lo)
    return xo, zo, po


@pytest.mark.parametrize("n", [1, 7, 63, 64, 65, 130, 256])
def test_pauli_mul_bit_exact(dev, n):
    api = _api()
    m = 3001
    xa, za, pa = synth.random_symplectic(m, n, seed=10 + n)
    xb, zb, pb = synth.random_symplectic(m, n, seed=20 + n)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64).reshape(-1)).to(dev)
    xo, zo, po = api.pauli_mul(n, t(xa), t(za), torch.from_numpy(pa).to(dev), t(xb), t(zb),
                               torch.from_numpy(pb).to(dev))
    rx, rz, rp = _oracle_mul(n, xa, za, pa, xb, zb, pb)
    np.testing.assert_array_equal(xo.cpu().numpy().view(np.uint64).reshape(m, -1), rx)
    np.testing.assert_array_equal(zo.cpu().numpy().view(np.uint64).reshape(m, -1), rz)
    np.testing.assert_array_equal(po.cpu().numpy(), rp)


def test_pauli_mul_in_place(dev):
    api = _api()
    n, m = 40, 500
    xa, za, pa = synth.random_symplectic(m, n, seed=1)
    xb, zb, pb = synth.random_symplectic(m, n, seed=2)
    ta = torch.from_numpy(xa.view(np.int64).reshape(-1)).to(dev)
    tz = torch.from_numpy(za.view(np.int64).reshape(-1)).to(dev)
    tp = torch.from_numpy(pa).to(dev)
    from paper_2606_28952_amd._abi import call
    from paper_2606_28952_amd.api import _ptr, _stream
    tb = [torch.from_numpy(v).to(dev) for v in (xb.view(np.int64).reshape(-1), zb.view(np.int64).reshape(-1), pb)]
    call("pbs_pauli_mul", n, m, _ptr(ta), _ptr(tz), _ptr(tp), _ptr(tb[0]), _ptr(tb[1]), _ptr(tb[2]),
         _ptr(ta), _ptr(tz), _ptr(tp), _stream())
    rx, rz, rp = _oracle_mul(n, xa, za, pa, xb, zb, pb)
    np.testing.assert_array_equal(ta.cpu().numpy().view(np.uint64).reshape(m, -1), rx)
    np.testing.assert_array_equal(tp.cpu().numpy(), rp)


def _canon_case(n, m, pool, seed, scale_spread):
    x, z, _ = synth.random_symplectic(m, n, seed=seed, pool=pool)
    rng = np.random.default_rng(seed + 1)
    mag = 10.0 ** rng.integers(-scale_spread, scale_spread + 1, size=m)
    c = (rng.standard_normal(m) * mag + 1j * rng.standard_normal(m) * mag).astype(np.complex128)
    # exact cancellations: duplicate some rows with negated coefficients
    k = m // 10
    x = np.concatenate([x, x[:k]])
    z = np.concatenate([z, z[:k]])
    c = np.concatenate([c, -c[:k]])
    return x, z, c


@pytest.mark.parametrize("n,m,pool,spread", [(5, 2000, 300, 0), (28, 50_000, 4000, 12), (64, 20_000, 20_000, 3),
                                             (130, 5000, 600, 20), (12, 1, 1, 0)])
@pytest.mark.parametrize("eps", [0.0, 1e-3, -1.0])
def test_canonicalize_bit_exact(dev, n, m, pool, spread, eps):
    api = _api()
    x, z, c = _canon_case(n, m, pool, seed=n + m, scale_spread=spread)
    s = api.PauliSum.create(n, x.reshape(-1), z.reshape(-1), c)
    s.canonicalize(eps)
    gx, gz, gc = s.read()
    rx, rz, rc = opauli.canonicalize_xz(x, z, c.real, c.imag, eps)
    np.testing.assert_array_equal(gx, rx)
    np.testing.assert_array_equal(gz, rz)
    assert gc.tobytes() == rc.tobytes()
    assert s.info()[2]


@pytest.mark.parametrize("m", [2047, 2048, 2049, 32768, 32769, 524288, 524289])
def test_canonicalize_at_scan_tile_boundaries(dev, m):
    """Contribution counts at the prefix sums' tile boundaries (2,048 items
    per tile; one single-block launch up to 16 tiles, three launches above):
    the head and survivor scans of the canonical reduction switch between
    the two forms at 32,768 items, and the radix sort's digit-count scan
    (256 counts per 4,096-key tile) at 524,288 keys; the result must stay
    bit-exact on both sides."""
    api = _api()
    x, z, _ = synth.random_symplectic(m, 40, seed=m, pool=max(1, m // 2))
    rng = np.random.default_rng(m + 1)
    c = (rng.standard_normal(m) + 1j * rng.standard_normal(m)).astype(np.complex128)
    s = api.PauliSum.create(40, x.reshape(-1), z.reshape(-1), c)
    s.canonicalize(0.0)
    gx, gz, gc = s.read()
    rx, rz, rc = opauli.canonicalize_xz(x, z, c.real, c.imag, 0.0)
    np.testing.assert_array_equal(gx, rx)
    np.testing.assert_array_equal(gz, rz)
    assert gc.tobytes() == rc.tobytes()


def _adversarial_segments():
    """Coefficient lists whose correctly rounded sums are decided by ties,
    tiny tails, cancellation or subnormals (one list per distinct string)."""
    t = 2.0 ** -53
    rng = np.random.default_rng(77)
    lists = [
        [1.0, t],                          # exact tie: rounds to even (1.0)
        [1.0, t, 2.0 ** -200],             # just above the tie: 1 + 2^-52
        [1.0, t, -(2.0 ** -200)],          # just below the tie: 1.0
        [-1.0, -t, -(2.0 ** -200)],        # mirrored
        [1e300, 1.0, -1e300],              # cancellation leaves 1.0
        [1e16, 1.0, -1e16, t],             # cancellation with a tail
        [2.0 ** -1074, 2.0 ** -1074, -(2.0 ** -1073)],  # subnormals summing to zero
        [2.0 ** -1074] * 3,                # subnormal sum
        [0.1] * 10,                        # classic rounding drift
        list(rng.standard_normal(5000) * 10.0 ** rng.integers(-8, 9, 5000)),  # long run
        [3.0, -3.0],                       # exact zero
    ]
    return lists


def test_canonicalize_adversarial_sums(dev):
    api = _api()
    n = 6
    lists = _adversarial_segments()
    rows, coeffs = [], []
    for k, vals in enumerate(lists):
        for j, v in enumerate(vals):
            rows.append(k)
            # imaginary parts reuse another list so both parts are exercised
            other = lists[(k + 3) % len(lists)]
            coeffs.append(complex(v, other[j % len(other)]))
    rows = np.array(rows)
    perm = np.random.default_rng(5).permutation(len(rows))
    rows = rows[perm]
    c = np.array(coeffs, dtype=np.complex128)[perm]
    x = (rows.astype(np.uint64) % 64).reshape(-1, 1)
    z = (rows.astype(np.uint64) // 64 + 1).reshape(-1, 1)
    s = api.PauliSum.create(n, x.reshape(-1), z.reshape(-1), c)
    s.canonicalize(0.0)
    gx, gz, gc = s.read()
    rx, rz, rc = opauli.canonicalize_xz(x, z, c.real, c.imag, 0.0)
    np.testing.assert_array_equal(gx, rx)
    np.testing.assert_array_equal(gz, rz)
    assert gc.tobytes() == rc.tobytes()


def test_canonicalize_empty(dev):
    api = _api()
    s = api.PauliSum.create(10, np.zeros(0, np.uint64), np.zeros(0, np.uint64), np.zeros(0, np.complex128))
    s.canonicalize()
    assert s.n_terms == 0


@pytest.mark.parametrize("n,ma,mb", [(4, 12, 9), (9, 40, 30), (70, 25, 20)])
def test_sum_mul_bit_exact(dev, n, ma, mb):
    api = _api()
    rng = np.random.default_rng(n)
    la, _ = synth.random_pauli_strings(ma, n, seed=100 + n)
    lb, _ = synth.random_pauli_strings(mb, n, seed=200 + n)
    ca = rng.standard_normal(ma) + 1j * rng.standard_normal(ma)
    cb = rng.standard_normal(mb) + 1j * rng.standard_normal(mb)
    A, B = OSum(n, la, ca), OSum(n, lb, cb)
    xa, za = opauli.letters_to_xz(la)
    xb, zb = opauli.letters_to_xz(lb)
    ga = api.PauliSum.create(n, xa.reshape(-1), za.reshape(-1), ca)
    gb = api.PauliSum.create(n, xb.reshape(-1), zb.reshape(-1), cb)
    gx, gz, gc = ga.mul(gb).read()
    rx, rz, rc = opauli.sum_product_canonical(A, B)
    np.testing.assert_array_equal(gx, rx)
    np.testing.assert_array_equal(gz, rz)
    assert gc.tobytes() == rc.tobytes()


def _jw_gpu(dev, h1, h2, e0=0.0, eps=0.0, eps_drop=0.0):
    api = _api()
    return api.jw_transform(torch.from_numpy(h1).to(dev), None if h2 is None else torch.from_numpy(h2).to(dev),
                            e0, eps, eps_drop).read()


def _assert_same(got, want):
    np.testing.assert_array_equal(got[0], want[0])
    np.testing.assert_array_equal(got[1], want[1])
    assert got[2].tobytes() == want[2].tobytes()


@pytest.mark.parametrize("n_o", [1, 2, 3, 6, 10, 14])
def test_jw_molecular_bit_exact(dev, n_o):
    h1, h2 = synth.molecular_spin_integrals(n_o, seed=1000 + n_o)
    got = _jw_gpu(dev, h1, h2)
    want = ojw.jw_hamiltonian(h1, h2)
    _assert_same(got, want)
    if n_o == 14:
        assert len(got[2]) == 55_371


def test_jw_hubbard_bit_exact(dev):
    h1, h2 = synth.hubbard_spin_integrals(4, 4)
    got = _jw_gpu(dev, h1, h2)
    _assert_same(got, ojw.jw_hamiltonian(h1, h2))
    assert len(got[2]) == 177


def test_jw_general_tensors_thresholds_e0(dev):
    rng = np.random.default_rng(7)
    n = 6
    h1 = rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.7)
    h2 = rng.standard_normal((n,) * 4) * (rng.random((n,) * 4) < 0.3)
    for eps, drop in [(0.0, 0.0), (0.5, 0.0), (0.0, 1e-2), (0.0, -1.0)]:
        _assert_same(_jw_gpu(dev, h1, h2, 1.25, eps, drop), ojw.jw_hamiltonian(h1, h2, 1.25, eps, drop))
    _assert_same(_jw_gpu(dev, h1, None, -0.5), ojw.jw_hamiltonian(h1, np.zeros((n,) * 4), -0.5))


def test_jw_multiword(dev):
    # 70 spin-orbitals: masks span two words
    n = 70
    rng = np.random.default_rng(8)
    h1 = np.zeros((n, n))
    for _ in range(60):
        p, q = rng.integers(0, n, 2)
        h1[p, q] += rng.standard_normal()
    h2 = np.zeros((n,) * 4)
    for _ in range(40):
        p, q, r, s = rng.integers(0, n, 4)
        h2[p, q, r, s] += rng.standard_normal()
    _assert_same(_jw_gpu(dev, h1, h2), ojw.jw_hamiltonian(h1, h2))


@pytest.mark.parametrize("n", [12, 130])
def test_sum_view_borrows_the_device_arrays(dev, n):
    """pbs_sum_view's pointers are the sum's own device arrays: a sum built
    from them through the C ABI reads back bit for bit, and an empty sum
    gives null pointers."""
    from ctypes import byref, c_void_p

    from paper_2606_28952_amd._abi import call

    api = _api()
    m = 517
    x, z, _ = synth.random_symplectic(m, n, seed=60 + n)
    rng = np.random.default_rng(61 + n)
    c = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    s = api.PauliSum.create(n, x.reshape(-1), z.reshape(-1), c)
    xp, zp, cp = s.view()
    assert xp and zp and cp
    out = c_void_p()
    call("pbs_sum_create", n, m, c_void_p(xp), c_void_p(zp), c_void_p(cp), None, byref(out))
    copy = api.PauliSum(out)
    for a, b in zip(s.read(), copy.read()):
        assert a.tobytes() == b.tobytes()
    empty = api.PauliSum.create(n, np.zeros(0, np.uint64), np.zeros(0, np.uint64), np.zeros(0, np.complex128))
    assert empty.view() == (0, 0, 0)
