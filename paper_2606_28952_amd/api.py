"""Python binding of the C ABI (argument marshalling only).

Bulk arrays are torch tensors on the HIP device; 64-bit masks travel as
torch.int64 tensors holding the unsigned bit patterns.  Every computation
runs in the HIP library on the current torch stream; handles free their
device memory when garbage-collected.
"""

import ctypes
from ctypes import byref, c_int32, c_uint32, c_uint64, c_void_p

import numpy as np
import torch

from . import _abi
from ._abi import PBS_C64, PBS_C128, call

__all__ = [
    "PauliSum", "Grouped", "Space", "pauli_mul", "jw_transform", "apply_pauli_sum", "expval", "expval_noalloc",
    "words_for", "PBS_C64", "PBS_C128", "KrylovPropagator", "Batch", "VQE", "MLP", "lbfgs_minimize",
    "STOP_REASONS",
]

STOP_REASONS = {0: "gradient", 1: "decrease", 2: "iterations", 3: "line search"}


def words_for(n_qubits):
    return max(1, (n_qubits + 63) // 64)


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        assert t.flags.c_contiguous
        return c_void_p(t.ctypes.data)
    assert t.is_contiguous(), "tensor must be contiguous"
    return c_void_p(t.data_ptr())


def _dev_u64(a, device="cuda"):
    """numpy uint64 / int64 / torch tensor -> contiguous int64 device tensor."""
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.int64).contiguous()
    arr = np.ascontiguousarray(np.asarray(a).astype(np.uint64).view(np.int64))
    return torch.from_numpy(arr).to(device)


def pauli_mul(n_qubits, xa, za, pa, xb, zb, pb):
    """Elementwise products of strings (device tensors); returns (x, z, phase)."""
    w = words_for(n_qubits)
    n = pa.numel()
    xo = torch.empty(n * w, dtype=torch.int64, device=xa.device)
    zo = torch.empty_like(xo)
    po = torch.empty(n, dtype=torch.uint8, device=xa.device)
    call("pbs_pauli_mul", n_qubits, n, _ptr(xa), _ptr(za), _ptr(pa), _ptr(xb), _ptr(zb), _ptr(pb),
         _ptr(xo), _ptr(zo), _ptr(po), _stream())
    return xo, zo, po


class PauliSum:
    """Handle to a library-owned Pauli sum (letter-form coefficients)."""

    def __init__(self, handle):
        self._h = c_void_p(handle) if not isinstance(handle, c_void_p) else handle

    @staticmethod
    def create(n_qubits, x, z, coeff):
        """x, z: uint64 words [m*W] (numpy host or torch device); coeff: complex [m]."""
        if isinstance(coeff, torch.Tensor):
            c = torch.view_as_real(coeff.to(torch.complex128).contiguous()).contiguous()
            xd, zd = _dev_u64(x, coeff.device), _dev_u64(z, coeff.device)
        else:
            c = np.ascontiguousarray(np.asarray(coeff, dtype=np.complex128).view(np.float64))
            xd = np.ascontiguousarray(np.asarray(x, dtype=np.uint64).reshape(-1))
            zd = np.ascontiguousarray(np.asarray(z, dtype=np.uint64).reshape(-1))
        m = (c.shape[0] // 2) if isinstance(c, np.ndarray) else c.shape[0]
        out = c_void_p()
        call("pbs_sum_create", n_qubits, m, _ptr(xd), _ptr(zd), _ptr(c), _stream(), byref(out))
        return PauliSum(out)

    def info(self):
        nq, nt, can = c_uint32(), c_uint64(), c_int32()
        call("pbs_sum_info", self._h, byref(nq), byref(nt), byref(can))
        return nq.value, nt.value, bool(can.value)

    @property
    def n_qubits(self):
        return self.info()[0]

    @property
    def n_terms(self):
        return self.info()[1]

    def read(self):
        """Host copies (x [m, W] uint64, z [m, W] uint64, coeff [m] complex128)."""
        nq, m, _ = self.info()
        w = words_for(nq)
        x = np.empty((m, w), np.uint64)
        z = np.empty((m, w), np.uint64)
        c = np.empty(m, np.complex128)
        call("pbs_sum_read", self._h, _ptr(x), _ptr(z), _ptr(c.view(np.float64)), _stream())
        return x, z, c

    def view(self):
        """Borrowed device pointers (x, z, coeff) as integers, valid until the
        sum is destroyed or canonicalized: x and z hold n_terms * W uint64
        words, coeff 2 * n_terms float64 (re, im); 0 for an empty sum."""
        nq, m = c_uint32(), c_uint64()
        x, z, c = c_void_p(), c_void_p(), c_void_p()
        call("pbs_sum_view", self._h, byref(nq), byref(m), byref(x), byref(z), byref(c))
        return x.value or 0, z.value or 0, c.value or 0

    def canonicalize(self, eps_drop=0.0):
        call("pbs_pauli_canonicalize", self._h, float(eps_drop), _stream())
        return self

    def mul(self, other, eps_drop=0.0):
        out = c_void_p()
        call("pbs_pauli_sum_mul", self._h, other._h, float(eps_drop), _stream(), byref(out))
        return PauliSum(out)

    def group(self):
        out = c_void_p()
        call("pbs_group_by_xmask", self._h, _stream(), byref(out))
        return Grouped(out)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _abi is not None and _abi._LIB is not None:
            _abi._LIB.pbs_sum_destroy(h)
            self._h = None


def jw_transform(h1, h2, e0=0.0, eps=0.0, eps_drop=0.0):
    """Canonical JW Hamiltonian from spin-orbital integrals (float64 device tensors)."""
    n = h1.shape[0]
    h1d = h1.to(dtype=torch.float64).contiguous()
    h2d = None if h2 is None else h2.to(dtype=torch.float64).contiguous()
    out = c_void_p()
    call("pbs_jw_transform", n, _ptr(h1d), _ptr(h2d), float(e0), float(eps), float(eps_drop), _stream(), byref(out))
    return PauliSum(out)


class Grouped:
    """Handle to an operator grouped by X-mask with its kernel tables."""

    def __init__(self, handle):
        self._h = handle

    def info(self):
        nq, g, m = c_uint32(), c_uint64(), c_uint64()
        call("pbs_grouped_info", self._h, byref(nq), byref(g), byref(m))
        return nq.value, g.value, m.value

    @property
    def n_groups(self):
        return self.info()[1]

    def read(self):
        """Host copies (xg [G], offsets [G+1], zk [M], ck [M] complex128)."""
        _, g, m = self.info()
        xg = np.empty(g, np.uint64)
        off = np.empty(g + 1, np.uint64)
        zk = np.empty(m, np.uint64)
        ck = np.empty(m, np.complex128)
        call("pbs_grouped_read", self._h, _ptr(xg), _ptr(off), _ptr(zk), _ptr(ck.view(np.float64)), _stream())
        return xg, off, zk, ck

    def factor(self, space):
        """Attaches spin-factorized phase tables for ``space``'s beta sector."""
        call("pbs_grouped_factor", self._h, space._h, _stream())
        return self

    def set_factored(self, mode):
        """True/7: all factor tables; False/0: none; otherwise a bit mask:
        1 the X_beta = 0 groups' rows, 2 the X_alpha = 0 class's move tables,
        4 the simple classes' alpha lists."""
        call("pbs_grouped_set_factored", self._h, 7 if mode is True else int(mode))
        return self

    def factor_info(self):
        """dict: tables present, factored X_beta = 0 groups and their largest
        rank, factored pair and quad groups of the X_alpha = 0 class and their
        ranks, and the N_beta of the tables."""
        info = np.zeros(11, np.uint32)
        call("pbs_grouped_factor_info", self._h, _ptr(info))
        keys = ["present", "zero_groups", "zero_max_rank", "pair_groups", "pair_rank", "quad_groups",
                "quad_rank", "n_beta", "alpha_lists", "n_alpha", "alpha_images"]
        return {k: int(v) for k, v in zip(keys, info)}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _abi is not None and _abi._LIB is not None:
            _abi._LIB.pbs_grouped_destroy(h)
            self._h = None


class Space:
    """Full 2^n space or a fixed-(N_alpha, N_beta) spin sector."""

    def __init__(self, handle):
        self._h = handle

    @staticmethod
    def full(n_qubits):
        out = c_void_p()
        call("pbs_space_full", n_qubits, byref(out))
        return Space(out)

    @staticmethod
    def sector(n_orb, n_alpha, n_beta):
        out = c_void_p()
        call("pbs_space_sector", n_orb, n_alpha, n_beta, _stream(), byref(out))
        return Space(out)

    @property
    def dim(self):
        d = c_uint64()
        call("pbs_space_dim", self._h, byref(d))
        return d.value

    def shape(self):
        vals = [c_uint32(), c_uint32(), c_uint32(), c_uint64(), c_uint64()]
        call("pbs_space_shape", self._h, *[byref(v) for v in vals])
        return tuple(v.value for v in vals)

    def rank(self, bits):
        """bits: int64 device tensor of basis patterns -> int64 indices (-1 outside)."""
        idx = torch.empty_like(bits, dtype=torch.int64)
        call("pbs_space_rank", self._h, bits.numel(), _ptr(bits), _ptr(idx), _stream())
        return idx

    def unrank(self, idx):
        bits = torch.empty_like(idx, dtype=torch.int64)
        call("pbs_space_unrank", self._h, idx.numel(), _ptr(idx), _ptr(bits), _stream())
        return bits

    def workspace_bytes(self):
        b = c_uint64()
        call("pbs_expval_workspace_bytes", self._h, byref(b))
        return b.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _abi is not None and _abi._LIB is not None:
            _abi._LIB.pbs_space_destroy(h)
            self._h = None


def _dtype_code(t):
    if t.dtype == torch.complex128:
        return PBS_C128
    if t.dtype == torch.complex64:
        return PBS_C64
    raise TypeError(f"state must be complex64 or complex128, got {t.dtype}")


def _check_states(space, psi, out):
    """The C ABI takes bare pointers: check lengths, dtypes and devices here."""
    code = _dtype_code(psi)
    if psi.device.type != "cuda" or psi.numel() != space.dim:
        raise ValueError(f"state must be a device vector of length {space.dim}")
    if out is not None and (out.dtype != psi.dtype or out.numel() != psi.numel() or out.device != psi.device):
        raise ValueError("out must match psi in dtype, length and device")
    return code


def apply_pauli_sum(grouped, space, psi, out=None):
    """out = P H P psi on the device (asynchronous on the current stream)."""
    _check_states(space, psi, out)
    if out is None:
        out = torch.empty_like(psi)
    call("pbs_apply_pauli_sum", grouped._h, space._h, _dtype_code(psi), _ptr(psi), _ptr(out), _stream())
    return out


def expval(grouped, space, psi, work=None, result=None, out=None):
    """(Re <psi|H|psi>, Im <psi|H|psi>, <psi|psi>) as a float64 device tensor of 3.
    With ``out`` the same pass also stores H psi there."""
    _check_states(space, psi, out)
    if work is None:
        work = torch.empty(max(1, space.workspace_bytes() // 8), dtype=torch.float64, device=psi.device)
    if result is None:
        result = torch.empty(3, dtype=torch.float64, device=psi.device)
    call("pbs_expval", grouped._h, space._h, _dtype_code(psi), _ptr(psi), _ptr(out), _ptr(result), _ptr(work),
         work.numel() * 8, _stream())
    return result


def expval_noalloc(grouped, space, psi, result, out=None):
    """expval with the library's fixed device workspace instead of a caller
    workspace; ``result`` (3 float64 on the device) is caller-owned, so the
    call itself allocates nothing.  Calls on one device must not overlap."""
    _check_states(space, psi, out)
    if result.dtype != torch.float64 or result.numel() < 3 or result.device != psi.device:
        raise ValueError("result must be a float64 device tensor of at least 3 values")
    call("pbs_expval_noalloc", grouped._h, space._h, _dtype_code(psi), _ptr(psi), _ptr(out), _ptr(result),
         _stream())
    return result


def _check_rows(space, psi, out, row_begin, row_end):
    """Host-side shape checks of a row-range call (the library checks the
    range itself against the sector)."""
    code = _dtype_code(psi)
    if psi.device.type != "cuda" or psi.numel() != space.dim:
        raise ValueError(f"state must be a device vector of length {space.dim}")
    dim_beta = space.shape()[4]
    rows = max(0, int(row_end) - int(row_begin))
    if out is not None and (out.dtype != psi.dtype or out.numel() != rows * dim_beta or out.device != psi.device):
        raise ValueError(f"out must hold {rows} x {dim_beta} values of psi's dtype on psi's device")
    return code, rows * dim_beta


def apply_pauli_sum_rows(grouped, space, psi, row_begin, row_end, out=None):
    """Alpha rows [row_begin, row_end) of P H P psi in a sector (one share of
    the target-row split), as a vector of (row_end - row_begin) * dim_beta."""
    code, n = _check_rows(space, psi, out, row_begin, row_end)
    if out is None:
        out = torch.empty(n, dtype=psi.dtype, device=psi.device)
    call("pbs_apply_pauli_sum_rows", grouped._h, space._h, code, _ptr(psi), _ptr(out), int(row_begin), int(row_end),
         _stream())
    return out


def expval_rows(grouped, space, psi, row_begin, row_end, work=None, result=None, out=None):
    """The share of alpha rows [row_begin, row_end) in expval's three sums;
    with ``out`` the same pass stores those rows of H psi."""
    code, n = _check_rows(space, psi, out, row_begin, row_end)
    if work is None:  # the share's partials: one per (row, 512-column chunk)
        dim_beta = space.shape()[4]
        rows = n // dim_beta if dim_beta else 0
        work = torch.empty(max(1, rows * ((dim_beta + 511) // 512) * 3), dtype=torch.float64, device=psi.device)
    if result is None:
        result = torch.empty(3, dtype=torch.float64, device=psi.device)
    call("pbs_expval_rows", grouped._h, space._h, code, _ptr(psi), _ptr(out), int(row_begin), int(row_end),
         _ptr(result), _ptr(work), work.numel() * 8, _stream())
    return result


class KrylovPropagator:
    """psi <- exp(-i H dt) psi by short-iterative Lanczos with m vectors; owns
    its device workspace (allocated once, reused by every step)."""

    def __init__(self, grouped, space, dtype=torch.complex64, m=12, device="cuda"):
        self.grouped, self.space, self.m = grouped, space, m
        self.code = PBS_C128 if dtype == torch.complex128 else PBS_C64
        nb = c_uint64()
        call("pbs_krylov_workspace_bytes", space._h, self.code, m, byref(nb))
        self.work = torch.empty(nb.value, dtype=torch.uint8, device=device)
        self.info = np.zeros(4, np.float64)

    def step(self, psi, dt):
        """Advances psi in place; returns (norm before, <H>, vectors used, last residual)."""
        if _dtype_code(psi) != self.code:
            raise TypeError("state dtype differs from the propagator's")
        call("pbs_krylov_step", self.grouped._h, self.space._h, self.code, _ptr(psi), float(dt), self.m,
             _ptr(self.work), self.work.numel(), _ptr(self.info), _stream())
        return tuple(float(v) for v in self.info)


class Batch:
    """One launch applying job i's operator to job i's state (spin sectors).

    jobs: list of (Grouped, Space, psi, out) with device state tensors of one
    dtype; the tensors must stay alive (the batch records their pointers)."""

    def __init__(self, jobs):
        n = len(jobs)
        self._keep = jobs
        code = _dtype_code(jobs[0][2])
        hs = (c_void_p * n)(*[j[0]._h.value for j in jobs])
        sps = (c_void_p * n)(*[j[1]._h.value for j in jobs])
        ps = (c_void_p * n)(*[j[2].data_ptr() for j in jobs])
        os_ = (c_void_p * n)(*[j[3].data_ptr() for j in jobs])
        for j in jobs:
            if _dtype_code(j[2]) != code or _dtype_code(j[3]) != code:
                raise TypeError("all batch states must share one dtype")
        out = c_void_p()
        call("pbs_batch_create", n, hs, sps, code, ps, os_, byref(out))
        self._h = out
        self.n = n

    def run(self, energies=None):
        """Applies every job; with a float64 device tensor of 3n, also writes
        each job's (Re E, Im E, <psi|psi>) from the same pass."""
        call("pbs_batch_run", self._h, _ptr(energies), _stream())
        return energies

    def set_config(self, config):
        """Job table for schedule bits ``config`` (PBS_BATCH_* in include/pbs.h)."""
        call("pbs_batch_set_config", self._h, int(config))

    def tune(self, reps=3):
        """Times every distinct schedule, keeps the fastest; returns (config, ms).
        Overwrites the outputs."""
        c, ms = c_uint32(), ctypes.c_double()
        call("pbs_batch_tune", self._h, int(reps), _stream(), byref(c), byref(ms))
        return c.value, ms.value

    def info(self):
        """(schedule bits in use, tuned ms per run or -1, workgroups per launch)."""
        c, ms, wg = c_uint32(), ctypes.c_double(), c_uint32()
        call("pbs_batch_info", self._h, byref(c), byref(ms), byref(wg))
        return c.value, ms.value, wg.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _abi is not None and _abi._LIB is not None:
            _abi._LIB.pbs_batch_destroy(h)
            self._h = None


class VQE:
    """Pauli-rotation ansatz R_{n-1} ... R_0 |ref>, R_k = exp(i theta_k P_k),
    on the full 2^(2 n_orb) space of a number-conserving grouped operator;
    energy and adjoint gradient on the device (float64)."""

    def __init__(self, grouped, n_orb, x, z, ref, dtype=torch.complex128):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.uint64).reshape(-1))
        z = np.ascontiguousarray(np.asarray(z, dtype=np.uint64).reshape(-1))
        if x.shape != z.shape:
            raise ValueError("x and z must have one word per rotation")
        self.n_rot = int(x.shape[0])
        self.n_orb = int(n_orb)
        self.dtype = dtype
        self._grouped = grouped  # keeps the operator alive
        code = PBS_C128 if dtype == torch.complex128 else PBS_C64
        out = c_void_p()
        call("pbs_vqe_create", grouped._h, self.n_orb, self.n_rot, _ptr(x), _ptr(z), int(ref), code, _stream(),
             byref(out))
        self._h = out

    def energy(self, theta):
        return self.energy_grad(theta, grad=False)[0]

    def energy_grad(self, theta, grad=True):
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1))
        if th.shape[0] != self.n_rot:
            raise ValueError(f"expected {self.n_rot} parameters")
        e = ctypes.c_double()
        g = np.zeros(self.n_rot, np.float64) if grad else None
        call("pbs_vqe_energy_grad", self._h, _ptr(th), byref(e), _ptr(g), _stream())
        return e.value, g

    def minimize(self, theta0, max_iter=500, g_tol=1e-6, f_tol=1e-12):
        """L-BFGS from theta0; returns (theta, energy, iterations, evaluations, reason)."""
        th = np.ascontiguousarray(np.asarray(theta0, dtype=np.float64).reshape(-1)).copy()
        if th.shape[0] != self.n_rot:
            raise ValueError(f"expected {self.n_rot} parameters")
        e, it, ev, why = ctypes.c_double(), c_uint32(), c_uint32(), c_int32()
        call("pbs_vqe_minimize", self._h, _ptr(th), int(max_iter), float(g_tol), float(f_tol), _stream(),
             byref(e), byref(it), byref(ev), byref(why))
        return th, e.value, it.value, ev.value, STOP_REASONS[why.value]

    def tune(self, reps=3):
        """Autotunes the batched sector launch (after an evaluation); (config, ms)."""
        c, ms = c_uint32(), ctypes.c_double()
        call("pbs_vqe_tune", self._h, int(reps), _stream(), byref(c), byref(ms))
        return c.value, ms.value

    def set_config(self, config):
        call("pbs_vqe_set_config", self._h, int(config))

    def set_groups(self, forward, adjoint):
        """Most rotations fused per forward / adjoint pass (1..3)."""
        call("pbs_vqe_set_groups", self._h, int(forward), int(adjoint))

    def blocks(self):
        """(sector blocks, blocks stored as sector (N_beta, N_alpha))."""
        nb, nt = c_uint32(), c_uint32()
        call("pbs_vqe_info", self._h, byref(nb), byref(nt))
        return nb.value, nt.value

    def state(self):
        psi = torch.empty(1 << (2 * self.n_orb), dtype=self.dtype, device="cuda")
        call("pbs_vqe_state", self._h, _ptr(psi), _stream())
        return psi

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _abi is not None and _abi._LIB is not None:
            _abi._LIB.pbs_vqe_destroy(h)
            self._h = None


_OBJECTIVE = ctypes.CFUNCTYPE(c_int32, c_void_p, c_uint32, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))


def lbfgs_minimize(fg, x0, max_iter=500, history=10, g_tol=1e-6, f_tol=1e-12):
    """L-BFGS of the library on a host objective fg(x) -> (f, g) over float64
    arrays; returns (x, f, iterations, evaluations, reason)."""
    x = np.ascontiguousarray(np.asarray(x0, dtype=np.float64).reshape(-1)).copy()
    n = x.shape[0]
    errors = []

    def trampoline(_user, m, xp, fp, gp):
        try:
            xv = np.ctypeslib.as_array(xp, shape=(m,)).copy()
            f, g = fg(xv)
            fp[0] = float(f)
            np.ctypeslib.as_array(gp, shape=(m,))[:] = np.asarray(g, dtype=np.float64).reshape(-1)
            return 0
        except Exception as exc:  # reported after the call returns
            errors.append(exc)
            return 1

    cb = _OBJECTIVE(trampoline)
    f, it, ev, why = ctypes.c_double(), c_uint32(), c_uint32(), c_int32()
    try:
        call("pbs_lbfgs_minimize", n, _ptr(x), ctypes.cast(cb, c_void_p), None, int(max_iter), int(history),
             float(g_tol), float(f_tol), byref(f), byref(it), byref(ev), byref(why))
    except _abi.PbsError:
        if errors:
            raise errors[0]
        raise
    return x, f.value, it.value, ev.value, STOP_REASONS[why.value]


class MLP:
    """Warm-start network 1 -> hidden -> hidden -> n_out (bf16 products, float32
    accumulation, Adam), parameters packed as in include/pbs.h."""

    def __init__(self, hidden, n_out, max_batch, params):
        self.hidden, self.n_out, self.max_batch = int(hidden), int(n_out), int(max_batch)
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
        if p.shape[0] != self.param_count(hidden, n_out):
            raise ValueError(f"expected {self.param_count(hidden, n_out)} parameters, got {p.shape[0]}")
        out = c_void_p()
        call("pbs_mlp_create", self.hidden, self.n_out, self.max_batch, _ptr(p), _stream(), byref(out))
        self._h = out

    @staticmethod
    def param_count(hidden, n_out):
        c = c_uint64()
        call("pbs_mlp_param_count", int(hidden), int(n_out), byref(c))
        return c.value

    def _rows(self, x):
        x = torch.as_tensor(x, dtype=torch.float32, device="cuda").reshape(-1).contiguous()
        return x, x.shape[0]

    def set_params(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
        call("pbs_mlp_set_params", self._h, _ptr(p), _stream())

    def params(self):
        p = np.zeros(self.param_count(self.hidden, self.n_out), np.float32)
        call("pbs_mlp_get_params", self._h, _ptr(p), _stream())
        return p

    def forward(self, x):
        x, n = self._rows(x)
        y = torch.empty((n, self.n_out), dtype=torch.float32, device="cuda")
        call("pbs_mlp_forward", self._h, n, _ptr(x), _ptr(y), _stream())
        return y

    def loss_grad(self, x, t):
        x, n = self._rows(x)
        t = torch.as_tensor(t, dtype=torch.float32, device="cuda").reshape(n, self.n_out).contiguous()
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        g = torch.empty(self.param_count(self.hidden, self.n_out), dtype=torch.float32, device="cuda")
        call("pbs_mlp_loss_grad", self._h, n, _ptr(x), _ptr(t), _ptr(loss), _ptr(g), _stream())
        return loss, g

    def train(self, x, t, n_steps, lr):
        losses = torch.empty(max(1, int(n_steps)), dtype=torch.float32, device="cuda")
        self.train_into(x, t, n_steps, lr, losses)
        return losses[:n_steps]

    def train_into(self, x, t, n_steps, lr, losses):
        """Training call writing the per-step losses into a caller buffer of
        at least n_steps floats (device); allocates nothing when x and t are
        contiguous float32 device tensors, so it can be graph-captured."""
        x, n = self._rows(x)
        t = torch.as_tensor(t, dtype=torch.float32, device="cuda").reshape(n, self.n_out).contiguous()
        if losses is not None and losses.numel() < int(n_steps):
            raise ValueError("losses buffer shorter than n_steps")
        call("pbs_mlp_train", self._h, n, _ptr(x), _ptr(t), int(n_steps), ctypes.c_float(lr),
             _ptr(losses) if losses is not None else None, _stream())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _abi is not None and _abi._LIB is not None:
            _abi._LIB.pbs_mlp_destroy(h)
            self._h = None
