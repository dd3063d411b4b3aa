"""The C-ABI library loads and exports every entry point include/hgsr.h
declares (no compute calls: CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hgsr.h")
LIB = os.path.join(ROOT, "paper_2507_15683_amd", "libhgsr.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hgsr_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2507_15683_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 15, syms
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2507_15683_amd import _lib
    assert set(_lib.SIGNATURES) == set(declared_symbols())


def test_version_and_error_strings(lib):
    lib.hgsr_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.hgsr_version()
    lib.hgsr_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.hgsr_last_error(), bytes)


def test_struct_layouts_match_header():
    """ctypes mirrors of the header structs have the C sizes (64-bit ABI)."""
    from paper_2507_15683_amd import _lib
    assert ctypes.sizeof(_lib.Gaussians) == 8 + 5 * 8 + 4 + 4 + 8 + 8 + 8 + 8  # n, 5 ptrs, deg, D, feat, parts...
    assert ctypes.sizeof(_lib.Intrinsics) == 24
    assert ctypes.sizeof(_lib.Opts) == 4 * 3 + 12 + 4 + 4 + 4 + 4
    assert ctypes.sizeof(_lib.TuneResult) == 20
    assert ctypes.sizeof(_lib.ResidualTargets) == 24
    assert ctypes.sizeof(_lib.Outputs) == 32
    assert ctypes.sizeof(_lib.Grads) == 7 * 8 + 8  # 7 pointers, render_id
    assert ctypes.sizeof(_lib.FeatureMaps) == 8 + 3 * 4 + 4   # pointer, width, height, layout, tail padding
    assert ctypes.sizeof(_lib.MatchMaps) == 4 * 8 + 3 * 4 + 4  # 4 pointers, D, width, height, tail padding
    assert ctypes.sizeof(_lib.MatchOut) == 7 * 8
    assert ctypes.sizeof(_lib.PnpProblem) == 4 * 8 + 4 * 4     # 2 ptrs, n, samples, n_hyp, tau, 2 counts
    assert ctypes.sizeof(_lib.PnpResult) == 6 * 8
    assert ctypes.sizeof(_lib.HostScene) == 8 + 5 * 8 + 4 + 4 + 8 + 4 + 4 + 8  # ..., n_parts, padding, offsets
    assert ctypes.sizeof(_lib.SlotUpload) == 24
    assert ctypes.sizeof(_lib.PcacheStats) == 4 * 4 + 3 * 8 + 4 + 4 + 8 + 8 + 4 + 4 + 64 * 24  # ..., upload[64]


# (ctypes mirror, C struct name) of every struct the binding passes by pointer
_MIRRORS = [("Gaussians", "hgsr_gaussians"), ("Intrinsics", "hgsr_intrinsics"), ("Opts", "hgsr_opts"),
            ("Outputs", "hgsr_outputs"), ("GradOutputs", "hgsr_grad_outputs"), ("Grads", "hgsr_grads"),
            ("RenderStats", "hgsr_render_stats"), ("TuneResult", "hgsr_tune_result"),
            ("ResidualTargets", "hgsr_residual_targets"), ("FeatureMaps", "hgsr_feature_maps"),
            ("MatchMaps", "hgsr_match_maps"), ("MatchOut", "hgsr_match_out"), ("PnpProblem", "hgsr_pnp_problem"),
            ("PnpResult", "hgsr_pnp_result"), ("HostScene", "hgsr_host_scene"), ("SlotUpload", "hgsr_slot_upload"),
            ("PcacheStats", "hgsr_pcache_stats")]


def test_struct_offsets_match_the_c_compiler(tmp_path):
    """Every field offset and struct size of the ctypes mirrors equals what
    the C compiler lays out from include/hgsr.h."""
    import subprocess
    from paper_2507_15683_amd import _lib
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hgsr.h"', 'int main(void) {']
    for py, c in _MIRRORS:
        lines.append(f'  printf("{py} size %zu\\n", sizeof({c}));')
        for f, _ in getattr(_lib, py)._fields_:
            lines.append(f'  printf("{py} {f} %zu\\n", offsetof({c}, {f}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        py, f, v = line.split()
        got[(py, f)] = int(v)
    for py, _ in _MIRRORS:
        cls = getattr(_lib, py)
        assert got[(py, "size")] == ctypes.sizeof(cls), py
        for f, _ in cls._fields_:
            assert got[(py, f)] == getattr(cls, f).offset, (py, f)


def test_invalid_arguments_rejected_on_host(lib):
    """Argument validation runs before anything touches a device."""
    from paper_2507_15683_amd import _lib
    L = _lib.load()
    # NULL ctx
    assert L.hgsr_render(None, None, None, 1, None, None, None, None) == 1
    assert L.hgsr_check_overflow(None, None, None) == 1
    assert L.hgsr_graph_launch(None, 1, None) == 5
    g = _lib.Gaussians()
    g.n = -1
    assert L.hgsr_validate(ctypes.byref(g), None) == 1
    g.n = 10
    assert L.hgsr_validate(ctypes.byref(g), None) == 1  # NULL arrays
    g2 = _lib.Gaussians()
    g2.n = 0
    g2.sh_degree = 4
    assert L.hgsr_validate(ctypes.byref(g2), None) == 1
    g2.sh_degree = 0
    g2.feat_dim = 12
    assert L.hgsr_validate(ctypes.byref(g2), None) == 1
    # significance scoring: NULL ctx, negative n, NULL outputs
    assert L.hgsr_significance(None, None, None, 1, None, None, None, None, None, None, None) == 1
    assert L.hgsr_significance_final(None, None, -1, None, None) == 1
    assert L.hgsr_significance_final(None, None, 5, None, None) == 1
    assert L.hgsr_significance_final(None, None, 0, None, None) == 0   # nothing to do
    # matching: NULL arguments, bad D, temperatures below 1/40
    assert L.hgsr_match(None, None, 0.1, 0.1, None, None) == 1
    mm = _lib.MatchMaps()
    mo = _lib.MatchOut()
    mm.D = 12
    assert L.hgsr_match(ctypes.c_void_p(1), ctypes.byref(mm), 0.1, 0.1, ctypes.byref(mo), None) == 1
    mm.D, mm.coarse_width, mm.coarse_height = 32, 4, 4
    mm.query_coarse = mm.render_coarse = 16
    assert L.hgsr_match(ctypes.c_void_p(1), ctypes.byref(mm), 0.01, 0.1, ctypes.byref(mo), None) == 1
    # pose solve, back-projection, consistency: argument checks
    assert L.hgsr_pnp(None, None, None, None, None, None) == 1
    pp = _lib.PnpProblem()
    pr = _lib.PnpResult()
    kk = _lib.Intrinsics(100.0, 100.0, 32.0, 24.0, 64, 48)
    pp.n, pp.n_hyp, pp.tau = 10, 0, 2.0
    assert L.hgsr_pnp(ctypes.c_void_p(1), ctypes.byref(pp), ctypes.byref(kk), ctypes.c_void_p(16),
                      ctypes.byref(pr), None) == 1   # NULL arrays / no samples
    assert L.hgsr_backproject(None, 64, 48, None, ctypes.byref(kk), None, 0, None, None) == 0   # nothing to do
    assert L.hgsr_backproject(None, 64, 48, None, ctypes.byref(kk), None, 5, None, None) == 1
    assert L.hgsr_pose_consistency(None, 3, 20.0, None, None, None) == 1
