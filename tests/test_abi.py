"""C ABI of libpond without a GPU: symbols, struct layout and argument checks.

Argument checks run before any HIP call, so every error path below is
exercised on the CPU with host pointers that are never dereferenced.
"""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_1806_05089_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pond.h")


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(pond_\w+)\s*\(", text, re.M)))


def test_header_declares_the_four_calls():
    names = _declared_functions()
    for n in ("pond_init", "pond_step", "pond_moments", "pond_step_adjoint", "pond_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (pond_\w+)", out))
    missing = [n for n in _declared_functions() if n not in exported]
    assert not missing, missing
    for n in _declared_functions():
        assert hasattr(lib, n)


def test_struct_layout_matches_header():
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "pond.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(pond_config), offsetof(pond_config, tau),
         offsetof(pond_config, eps_rel), sizeof(pond_state), sizeof(pond_stats));
  printf("%zu\n", offsetof(pond_stats, mean_iters));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        cfile = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(cfile, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), cfile, "-o", exe], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True,
                                                check=True).stdout.split()]
    assert vals[0] == C.sizeof(_lib.pond_config)
    assert vals[1] == _lib.pond_config.tau.offset
    assert vals[2] == _lib.pond_config.eps_rel.offset
    assert vals[3] == C.sizeof(_lib.pond_state)
    assert vals[4] == C.sizeof(_lib.pond_stats)
    assert vals[5] == _lib.pond_stats.mean_iters.offset


def test_abi_version(lib):
    assert lib.pond_abi_version() == 101


def _cfg(**kw):
    base = dict(nx=8, ny=8, q1d=4, precision=0, isothermal=0, bc_x=0, bc_y=0, max_iter=20,
                fixed_iter=0, seed_mode=0, tau=0.6, eps_abs=1e-12, eps_rel=1e-10)
    base.update(kw)
    return _lib.pond_config(*[base[f] for f, _ in _lib.pond_config._fields_])


# host buffers standing in for device pointers: never touched, checks fail first
_BUF = (C.c_double * 4096)()
_BUF2 = (C.c_double * 4096)()


def _state(f, g, iters=None):
    return _lib.pond_state(C.addressof(f) if f is not None else None,
                           C.addressof(g) if g is not None else None,
                           C.addressof(iters) if iters is not None else None)


@pytest.mark.parametrize("bad,code", [
    (dict(nx=0), _lib.POND_E_INVALID), (dict(ny=-3), _lib.POND_E_INVALID),
    (dict(q1d=5), _lib.POND_E_INVALID), (dict(precision=7), _lib.POND_E_INVALID),
    (dict(isothermal=2), _lib.POND_E_INVALID), (dict(bc_x=3), _lib.POND_E_INVALID),
    (dict(max_iter=0), _lib.POND_E_INVALID), (dict(max_iter=64), _lib.POND_E_INVALID),
    (dict(fixed_iter=-1), _lib.POND_E_INVALID), (dict(seed_mode=3), _lib.POND_E_INVALID),
    (dict(tau=0.0), _lib.POND_E_INVALID), (dict(tau=float("nan")), _lib.POND_E_INVALID),
    (dict(eps_abs=-1.0), _lib.POND_E_INVALID),
])
def test_step_rejects_bad_config(lib, bad, code):
    cfg = _cfg(**bad)
    sin, sout = _state(_BUF, _BUF2), _state(_BUF2, _BUF)
    rc = lib.pond_step(C.byref(cfg), C.byref(sin), C.byref(sout), 1, None, None)
    assert rc == code
    assert len(lib.pond_last_error()) > 0


def test_null_and_alias_checks(lib):
    cfg = _cfg(nx=4, ny=4)
    f1 = (C.c_double * (16 * 16))()
    g1 = (C.c_double * (3 * 16))()
    f2 = (C.c_double * (16 * 16))()
    g2 = (C.c_double * (3 * 16))()
    assert lib.pond_step(None, None, None, 1, None, None) == _lib.POND_E_NULL
    s_in = _state(f1, g1)
    s_null = _state(None, g2)
    assert lib.pond_step(C.byref(cfg), C.byref(s_in), C.byref(s_null), 1, None, None) == _lib.POND_E_NULL
    s_alias = _state(f1, g2)
    assert lib.pond_step(C.byref(cfg), C.byref(s_in), C.byref(s_alias), 1, None, None) == _lib.POND_E_ALIAS
    s_cross = _state(f2, g1)  # output g aliases input g
    assert lib.pond_step(C.byref(cfg), C.byref(s_in), C.byref(s_cross), 1, None, None) == _lib.POND_E_ALIAS
    s_out = _state(f2, g2)
    assert lib.pond_step(C.byref(cfg), C.byref(s_in), C.byref(s_out), 0, None, None) == _lib.POND_E_INVALID
    assert lib.pond_moments(C.byref(cfg), None, None, None, None, None, None, None) == _lib.POND_E_NULL
    assert lib.pond_init(C.byref(cfg), None, None, None, None, C.byref(s_out), None) == _lib.POND_E_NULL
    # adjoint needs the forward pass counts
    a_out = _state(f2, g2)
    assert lib.pond_step_adjoint(C.byref(cfg), C.byref(s_in), C.byref(s_in), C.byref(a_out),
                                 C.byref(a_out), None, None) == _lib.POND_E_NULL
    # recorded steps: the tape, and the output's pass counts, are required
    assert lib.pond_tape_bytes(C.byref(cfg), None) == _lib.POND_E_NULL
    tape = (C.c_uint8 * 4096)()
    assert lib.pond_step_record(C.byref(cfg), C.byref(s_in), C.byref(s_out), None,
                                None) == _lib.POND_E_NULL
    assert lib.pond_step_record(C.byref(cfg), C.byref(s_in), C.byref(s_out), tape,
                                None) == _lib.POND_E_NULL  # s_out.iters is NULL
    assert lib.pond_step_adjoint_recorded(C.byref(cfg), C.byref(s_in), C.byref(s_in), None,
                                          C.byref(a_out), C.byref(a_out), None,
                                          None) == _lib.POND_E_NULL


def test_tape_bytes(lib):
    """((K + 1) * 4 + q^2) * nx * ny doubles, K = fixed_iter or max_iter."""
    n = C.c_int64(0)
    cfg = _cfg(nx=10, ny=6, max_iter=20)
    assert lib.pond_tape_bytes(C.byref(cfg), C.byref(n)) == _lib.POND_OK
    assert n.value == (21 * 4 + 16) * 60 * 8
    cfg = _cfg(nx=10, ny=6, q1d=3, fixed_iter=3)
    assert lib.pond_tape_bytes(C.byref(cfg), C.byref(n)) == _lib.POND_OK
    assert n.value == (4 * 4 + 9) * 60 * 8
    cfg = _cfg(nx=10, ny=6, max_iter=0)
    assert lib.pond_tape_bytes(C.byref(cfg), C.byref(n)) == _lib.POND_E_INVALID


def test_python_binding_fails_loudly_without_library(tmp_path):
    with pytest.raises(ImportError):
        _lib._lib_saved = _lib._lib
        try:
            _lib._lib = None
            _lib.load(str(tmp_path / "missing.so"))
        finally:
            _lib._lib = _lib._lib_saved
