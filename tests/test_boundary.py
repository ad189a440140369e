"""The C ABI without a GPU: exported symbols, struct layouts, host-side calls."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2602_17950_amd import gs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gs.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\**\s*(gs_[a-z_0-9]+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 12
    lib = gs.load()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(gs.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", gs.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (gs_[a-z_0-9]+)$", out, flags=re.M))
    assert set(names) <= exported


def test_struct_layouts_match_header(tmp_path):
    """sizeof/offsetof of the C structs (compiled against gs.h) equal the ctypes mirrors."""
    structs = {"gs_grid": gs.gs_grid, "gs_trap": gs.gs_trap, "gs_params": gs.gs_params,
               "gs_options": gs.gs_options, "gs_result": gs.gs_result, "gs_request": gs.gs_request}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(src)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split("\n") if l)
    for name, cls in structs.items():
        assert int(got[name]) == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)


def test_default_options_and_footprint():
    o = gs.default_options()
    assert o.stop_kind == gs.GS_STOP_ENERGY and o.tol == 1e-12 and o.precision == gs.GS_FP64
    assert o.theta_trial == 0.1 and o.sigma == 0.5 and o.max_backtrack == 40
    from paper_2602_17950_amd import inputs
    pb = inputs.Problem(dim=2, n=(256, 256), L=(12.0, 12.0))
    b64 = gs.footprint_bytes(pb, gs.GS_FP64)
    b32 = gs.footprint_bytes(pb, gs.GS_FP32)
    M = 256 * 256
    field = 3 * M * 16
    # 8 working fields + 8 scratch fields + the P_V factors, plus reduction rows
    assert field * 16 + 3 * M * 8 <= b64 <= field * 16 + 3 * M * 8 + 2 * 2 ** 20
    assert field * 8 + 3 * M * 4 <= b32 <= field * 8 + 3 * M * 4 + 2 * 2 ** 20
    assert gs.footprint_bytes(pb, gs.GS_MIXED) == b64 + b32
    # double state, float direction: r^n, r^{n-1}, Pr, P, H_L P^, u and the P_V factors halve
    bmx = gs.footprint_bytes(pb, gs.GS_FP64, dir_precision=gs.GS_FP32)
    assert abs(b64 - bmx - (6 * field // 2 + 3 * M * 4)) <= 2 ** 20   # reduction rows differ slightly
    assert gs.footprint_bytes(pb, gs.GS_MIXED, dir_precision=gs.GS_FP32) == bmx + b32
    assert gs.footprint_bytes(pb, gs.GS_FP64, dir_precision=7) == 0
    # the options are validated: preconditioner kind and stopping criterion
    assert gs.footprint_bytes(pb, gs.GS_FP64, precond=gs.GS_PC_POTENTIAL) == b64
    assert gs.footprint_bytes(pb, gs.GS_FP64, precond=3) == 0
    assert gs.footprint_bytes(pb, gs.GS_FP64, stop_kind=gs.GS_STOP_WAVEFN) == b64
    assert gs.footprint_bytes(pb, gs.GS_FP64, stop_kind=4) == 0
    assert gs.footprint_bytes(pb, gs.GS_FP64, line_search=gs.GS_LS_EXACT) == b64
    assert gs.footprint_bytes(pb, gs.GS_FP64, line_search=2) == 0
    # lengths 3 * 2^a are supported, other factors are not
    assert gs.footprint_bytes(inputs.Problem(dim=2, n=(96, 48), L=(12.0, 12.0)), gs.GS_FP64) > 0
    assert gs.footprint_bytes(inputs.Problem(dim=2, n=(12, 64), L=(12.0, 12.0)), gs.GS_FP64) == 0
    bad = inputs.Problem(dim=2, n=(40, 64), L=(12.0, 12.0))
    assert gs.footprint_bytes(bad, gs.GS_FP64) == 0
    pb3 = inputs.Problem(dim=3, n=(128, 128, 128), L=(8.0, 8.0, 8.0))
    M3 = 128 ** 3
    assert gs.footprint_bytes(pb3, gs.GS_FP64) >= 3 * M3 * 16 * 16 + 3 * M3 * 8


def test_errors_without_device():
    """Argument validation happens before any device work."""
    lib = gs.load()
    g = gs.make_grid(2, (64, 64), (8.0, 8.0))
    o = gs.default_options()
    rc = lib.gs_solve(None, C.byref(g), None, None, C.byref(o), None, None, None)
    assert rc == gs.GS_EINVAL
    assert "NULL" in gs.last_error()
    rc = lib.gs_kernel_timer_start(None, 0)
    assert rc == gs.GS_EINVAL
    q = gs.gs_request()
    t = C.c_uint64()
    assert lib.gs_submit(None, C.byref(q), C.byref(t)) == gs.GS_EINVAL
    assert lib.gs_poll(None, 1, None) == gs.GS_EINVAL
    assert lib.gs_wait(None, 1, None) == gs.GS_EINVAL
    assert lib.gs_cancel(None, 1) == gs.GS_EINVAL
    assert lib.gs_progress(None, 0) == gs.GS_EINVAL
    assert lib.gs_batch_solve(None, 1, C.byref(q), None) == gs.GS_EINVAL
    assert lib.gs_set_hbm_budget(None, 0) == gs.GS_EINVAL
    assert lib.gs_memory_stats(None, None, None, None) == gs.GS_EINVAL
