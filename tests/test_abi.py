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
  printf("%zu %zu\n", offsetof(pond_stats, mean_iters), offsetof(pond_stats, iter_hist));
  printf("%d %d\n", (int)POND_OP_STEP, (int)POND_OP_STEP_ADJOINT);
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
    assert vals[6] == _lib.pond_stats.iter_hist.offset
    assert C.sizeof(_lib.pond_stats) == _lib.pond_stats.iter_hist.offset + 64 * 8
    assert vals[7:9] == [_lib.POND_OP_STEP, _lib.POND_OP_STEP_ADJOINT]


def test_abi_version(lib):
    assert lib.pond_abi_version() == 201


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
    ws = (C.c_uint8 * 4096)()
    assert lib.pond_step_adjoint(C.byref(cfg), C.byref(s_in), C.byref(s_in), C.byref(a_out),
                                 C.byref(a_out), None, ws, 4096, None) == _lib.POND_E_NULL
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


def test_workspace_bytes(lib):
    """POND_OP_STEP needs none; the adjoint's is the tape plus one state, each
    part rounded up to 256 bytes."""
    n = C.c_int64(-1)
    cfg = _cfg(nx=10, ny=6, max_iter=20)
    assert lib.pond_workspace_bytes(C.byref(cfg), _lib.POND_OP_STEP, C.byref(n)) == _lib.POND_OK
    assert n.value == 0
    assert lib.pond_workspace_bytes(C.byref(cfg), _lib.POND_OP_STEP_ADJOINT,
                                    C.byref(n)) == _lib.POND_OK
    up = lambda b: (b + 255) // 256 * 256
    tape = (21 * 4 + 16) * 60 * 8
    assert n.value == up(tape) + up(16 * 60 * 8) + up(3 * 60 * 8) + up(60)
    cfg32 = _cfg(nx=10, ny=6, precision=1, fixed_iter=2)
    assert lib.pond_workspace_bytes(C.byref(cfg32), _lib.POND_OP_STEP_ADJOINT,
                                    C.byref(n)) == _lib.POND_OK
    assert n.value == up((3 * 4 + 16) * 60 * 8) + up(16 * 60 * 4) + up(3 * 60 * 8) + up(60)
    assert lib.pond_workspace_bytes(C.byref(cfg), 7, C.byref(n)) == _lib.POND_E_INVALID
    assert lib.pond_workspace_bytes(C.byref(cfg), _lib.POND_OP_STEP, None) == _lib.POND_E_NULL


def test_adjoint_workspace_checks(lib):
    """Missing, too small, misaligned or overlapping workspace: rejected before
    any launch."""
    cfg = _cfg(nx=4, ny=4, fixed_iter=2)
    f1, g1 = (C.c_double * 256)(), (C.c_double * 48)()
    f2, g2 = (C.c_double * 256)(), (C.c_double * 48)()
    f3, g3 = (C.c_double * 256)(), (C.c_double * 48)()
    it = (C.c_uint8 * 16)()
    s_in, s_fwd = _state(f1, g1), _state(f2, g2, it)
    a_out, a_in = _state(f2, g2), _state(f3, g3)
    need = C.c_int64(0)
    assert lib.pond_workspace_bytes(C.byref(cfg), _lib.POND_OP_STEP_ADJOINT,
                                    C.byref(need)) == _lib.POND_OK
    ws = (C.c_uint8 * (need.value + 64))()
    base = C.addressof(ws)
    aligned = (base + 15) // 16 * 16
    call = lambda p, n: lib.pond_step_adjoint(C.byref(cfg), C.byref(s_in), C.byref(s_fwd),
                                              C.byref(a_out), C.byref(a_in), None, p, n, None)
    assert call(None, need.value) == _lib.POND_E_NULL
    assert call(aligned, need.value - 1) == _lib.POND_E_INVALID
    assert call(aligned + 8, need.value) == _lib.POND_E_INVALID
    assert "workspace" in lib.pond_last_error().decode()
    # workspace over the input state
    big = (C.c_uint8 * (need.value + 4096))()
    s_in_over = _lib.pond_state((C.addressof(big) + 15) // 16 * 16, C.addressof(g1), None)
    assert lib.pond_step_adjoint(C.byref(cfg), C.byref(s_in_over), C.byref(s_fwd),
                                 C.byref(a_out), C.byref(a_in), None,
                                 (C.addressof(big) + 15) // 16 * 16, need.value,
                                 None) == _lib.POND_E_ALIAS


def test_fp32_mixed_adaptive_rejects_fp64_tolerances(lib):
    """The paper's FP64 tolerances are below FP32 resolution: an adaptive
    FP32-mixed step with them is refused (fixed passes need no test)."""
    f1, g1 = (C.c_float * 256)(), (C.c_double * 48)()
    f2, g2 = (C.c_float * 256)(), (C.c_double * 48)()
    s_in, s_out = _state(f1, g1), _state(f2, g2)
    cfg = _cfg(nx=4, ny=4, precision=1)
    assert lib.pond_step(C.byref(cfg), C.byref(s_in), C.byref(s_out), 1, None,
                         None) == _lib.POND_E_INVALID
    assert "2^-23" in lib.pond_last_error().decode()
    tape = (C.c_uint8 * 8192)()
    it = (C.c_uint8 * 16)()
    s_out_it = _state(f2, g2, it)
    assert lib.pond_step_record(C.byref(cfg), C.byref(s_in), C.byref(s_out_it), tape,
                                None) == _lib.POND_E_INVALID


def test_init_adjoint_checks(lib):
    cfg = _cfg(nx=4, ny=4)
    af, ag = (C.c_double * 256)(), (C.c_double * 48)()
    assert lib.pond_init_adjoint(C.byref(cfg), None, ag, None, None, None, None,
                                 None) == _lib.POND_E_NULL
    # adj_rho inside adj_f
    assert lib.pond_init_adjoint(C.byref(cfg), af, ag, C.addressof(af) + 64, None, None, None,
                                 None) == _lib.POND_E_ALIAS
    bad = _cfg(nx=4, ny=4, q1d=2)
    out = (C.c_double * 16)()
    assert lib.pond_init_adjoint(C.byref(bad), af, ag, out, None, None, None,
                                 None) == _lib.POND_E_INVALID


def test_step_noalloc_argument_checks(lib):
    """pond_step_noalloc checks like pond_step, and refuses a grid whose step
    tiles exceed its fixed scratch, before any HIP call."""
    f1, g1 = (C.c_double * 256)(), (C.c_double * 48)()
    f2, g2 = (C.c_double * 256)(), (C.c_double * 48)()
    s_in, s_out = _state(f1, g1), _state(f2, g2)
    cfg = _cfg(nx=4, ny=4)
    assert lib.pond_step_noalloc(C.byref(cfg), C.byref(s_in), None, 1, None,
                                 None) == _lib.POND_E_NULL
    s_alias = _state(f1, g2)
    assert lib.pond_step_noalloc(C.byref(cfg), C.byref(s_in), C.byref(s_alias), 1, None,
                                 None) == _lib.POND_E_ALIAS
    assert lib.pond_step_noalloc(C.byref(cfg), C.byref(s_in), C.byref(s_out), 0, None,
                                 None) == _lib.POND_E_INVALID
    # 4096 x 4100 in FP32-mixed: 128 x 513 tiles of 32 x 8 > 65,536
    big = _cfg(nx=4096, ny=4100, precision=1, eps_abs=1e-6, eps_rel=1e-5)
    assert lib.pond_step_noalloc(C.byref(big), C.byref(s_in), C.byref(s_out), 1, None,
                                 None) == _lib.POND_E_INVALID
    assert "scratch" in lib.pond_last_error().decode()
    # D2Q9 in FP64 steps on 32 x 8 tiles too; D2Q16 FP64 on 32 x 16 fits
    big9 = _cfg(nx=4096, ny=4100, q1d=3)
    assert lib.pond_step_noalloc(C.byref(big9), C.byref(s_in), C.byref(s_out), 1, None,
                                 None) == _lib.POND_E_INVALID
    assert "scratch" in lib.pond_last_error().decode()
