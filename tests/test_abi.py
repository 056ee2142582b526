"""The C-ABI library loads and exports every symbol include/pbs.h declares,
and its host-side argument checks return the documented status codes.  No
call here touches a GPU."""

import ctypes
import os
import re
from ctypes import byref, c_uint64, c_void_p

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pbs.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pbs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2606_28952_amd import _abi

    if not os.path.exists(_abi.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    return _abi.lib()


def test_header_declares_the_core_calls():
    names = set(_declared())
    for fn in ["pbs_pauli_mul", "pbs_pauli_canonicalize", "pbs_jw_transform", "pbs_group_by_xmask",
               "pbs_apply_pauli_sum", "pbs_expval", "pbs_krylov_step", "pbs_batch_tune", "pbs_vqe_energy_grad",
               "pbs_mlp_train", "pbs_lbfgs_minimize"]:
        assert fn in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2606_28952_amd import _abi

    declared = _declared()
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(lib, name), name
    # the binding declares exactly the header's functions
    assert sorted(_abi.SIGNATURES) == declared


def test_abi_version(lib):
    assert lib.pbs_abi_version() == 1


def test_host_side_errors(lib):
    from paper_2606_28952_amd import _abi

    out = c_void_p()
    assert lib.pbs_space_full(0, byref(out)) == 2          # ERR_RANGE
    assert b"1..40" in lib.pbs_last_error()
    assert lib.pbs_space_full(41, byref(out)) == 2
    assert lib.pbs_space_sector(40, 1, 1, None, byref(out)) == 2
    assert lib.pbs_space_sector(5, 6, 1, None, byref(out)) == 1   # more electrons than orbitals
    assert lib.pbs_sum_info(None, None, None, None) == 1
    assert lib.pbs_sum_view(None, None, None, None, None, None) == 1
    assert lib.pbs_apply_pauli_sum(None, None, 0, None, None, None) == 1
    assert lib.pbs_apply_pauli_sum_rows(None, None, 0, None, None, 0, 1, None) == 1
    assert lib.pbs_expval_rows(None, None, 0, None, None, 0, 1, None, None, 0, None) == 1
    assert lib.pbs_jw_transform(0, None, None, 0.0, 0.0, 0.0, None, byref(out)) == 2
    assert lib.pbs_jw_transform(4, None, None, 0.0, 0.0, 0.0, None, byref(out)) == 1
    assert lib.pbs_pauli_mul(300, 1, *([None] * 9), None) == 2
    assert lib.pbs_pauli_mul(10, 0, *([None] * 9), None) == 0      # empty input is a no-op
    assert lib.pbs_group_by_xmask(None, None, byref(out)) == 1
    assert lib.pbs_last_error() != b""


def test_full_space_handle_without_device(lib):
    out = c_void_p()
    assert lib.pbs_space_full(12, byref(out)) == 0
    dim = c_uint64()
    assert lib.pbs_space_dim(out, byref(dim)) == 0 and dim.value == 4096
    nb = c_uint64()
    assert lib.pbs_expval_workspace_bytes(out, byref(nb)) == 0 and nb.value == 16 * 3 * 8
    # a full space has no sector shape
    assert lib.pbs_space_shape(out, None, None, None, None, None) == 1
    lib.pbs_space_destroy(out)
    assert lib.pbs_last_error() == b"not a sector space"


def test_binding_raises_when_library_missing(monkeypatch, tmp_path):
    from paper_2606_28952_amd import _abi

    monkeypatch.setattr(_abi, "_LIB", None)
    monkeypatch.setattr(_abi, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        _abi.lib()
