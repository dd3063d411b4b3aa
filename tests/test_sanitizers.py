"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the oracle's C++ built with both and driven through its Python
wrappers (brute-force and tiled renders, tile lists, the frozen renderer,
the contribution walk, the projection dump, SH and box helpers) on ragged
tiny scenes, and the library's host-only C++ (partition boxes and plan, the
slot policy, the spatial order) driven by a C++ test program.  Any sanitizer
report aborts the child process and fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _runtime(name):
    p = subprocess.check_output(["g++", f"-print-file-name={name}"], text=True).strip()
    if not os.path.isabs(p) or not os.path.exists(p):
        pytest.skip(f"{name} not found for g++")
    return p


DRIVER = r'''
import numpy as np, oracle, synth
for seed in range(6):
    n = 40 + 29 * seed
    sc, P, cam = synth.tiny_scene(n, 500 + seed, width=37 + 7 * seed, height=29 + 5 * seed,
                                  sh_degree=seed % 4, feat_dim=(0, 8, 16, 32, 64, 8)[seed])
    a = oracle.render(sc, P[0], cam, mode="brute")
    for tile in (8, 16, 32):
        b = oracle.render(sc, P[0], cam, mode="tiled", tile=tile, want_lists=True, list_cap=64)
        assert np.array_equal(a["rgb"], b["rgb"])
        off, ids, edge = oracle.tile_lists(sc, P[0], cam, tile=tile)
    fr = oracle.render_frozen(sc, P[0], cam, b["lists"], b["nblend"])
    assert np.allclose(fr["rgb"], b["rgb"], atol=1e-12)
    oracle.project(sc, P[0], cam)
    oracle.contrib(sc, P[0], cam)
empty = sc.subset(np.zeros(0, dtype=np.int64))
oracle.render(empty, P[0], cam)
oracle.sh_basis(3, np.random.default_rng(0).normal(size=(50, 3)))
print("oracle under sanitizers ok")
'''


def test_oracle_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["g++", *SAN, "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                           "-o", lib, os.path.join(ROOT, "oracle", "hgsr_oracle.cpp")])
    env = dict(os.environ, HGSR_ORACLE_LIB=lib, LD_PRELOAD=_runtime("libasan.so") + ":" + _runtime("libubsan.so"),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", DRIVER], env=env, cwd=ROOT, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "oracle under sanitizers ok" in r.stdout


def test_host_code_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_driver")
    subprocess.check_call(["g++", *SAN, "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
                           os.path.join(ROOT, "paper_2507_15683_amd", "csrc", "host.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="abort_on_error=1"))
    assert r.returncode == 0, r.stderr[-4000:]
    assert "host driver ok" in r.stdout
