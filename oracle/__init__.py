"""FP64 CPU oracle of the Gaussian-splat renderer -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its Python
binding) never imports, links or calls it, and the two share no code.

The arithmetic lives in `hgsr_oracle.cpp` (plain C++, double precision,
OpenMP over tiles/rows); this module marshals numpy arrays to it.  The pose
exponential and the refinement residual used by the finite-difference checks
are in `se3.py` and `loss.py`; significance scoring with the render
visibility check is in `significance.py`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hgsr_oracle.cpp")
# HGSR_ORACLE_LIB names another build of the same source (the sanitizer test
# loads an AddressSanitizer/UBSan build through it).
_LIB = os.environ.get("HGSR_ORACLE_LIB", os.path.join(_HERE, "liboracle.so"))


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (IEEE double semantics: no fast-math, no FMA
    contraction, so the brute-force and tiled renderers agree bit for bit)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-o", _LIB + ".tmp", _SRC]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Scene(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacities", ctypes.c_void_p), ("sh", ctypes.c_void_p),
                ("sh_degree", ctypes.c_int32), ("feat_dim", ctypes.c_int32), ("feat", ctypes.c_void_p),
                ("means64", ctypes.c_void_p), ("opac64", ctypes.c_void_p), ("log_scales64", ctypes.c_void_p),
                ("quats64", ctypes.c_void_p), ("sh64", ctypes.c_void_p), ("feat64", ctypes.c_void_p)]


class _Camera(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("near_z", ctypes.c_double), ("bg", ctypes.c_double * 3)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.orc_project.argtypes = [P, P, P, P, P]
        lib.orc_render.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32] + [P] * 9 + [ctypes.c_int32]
        lib.orc_render_frozen.argtypes = [P, P, P, P, P, ctypes.c_int32, P, P, P, P, P]
        lib.orc_tile_lists.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_double, P, P, ctypes.c_int64, P, P]
        lib.orc_sh_basis.argtypes = [ctypes.c_int32, P, ctypes.c_int64, P]
        lib.orc_min_q_box.argtypes = [P, ctypes.c_int64, P]
        lib.orc_contrib.argtypes = [P, P, P, ctypes.c_int32, P, P, P]
        lib.orc_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class _Bound:
    """Keeps the numpy arrays referenced by a ctypes struct alive."""

    def __init__(self, scene, cam, near=0.2, bg=(0.0, 0.0, 0.0), overrides=None):
        c = lambda a, dt: np.ascontiguousarray(a, dtype=dt)
        ov = overrides or {}
        self.ov = {k: c(ov[k], np.float64) for k in ("means", "opacities", "log_scales", "quats", "sh", "feat")
                   if ov.get(k) is not None}
        self.arrays = [c(scene.means, np.float32), c(scene.log_scales, np.float32), c(scene.quats, np.float32),
                       c(scene.opacities, np.float32), c(scene.sh, np.float32)]
        self.feat = None if scene.feat is None else c(scene.feat, np.uint16)
        m, ls, q, o, sh = self.arrays
        self.s = _Scene(scene.means.shape[0], m.ctypes.data, ls.ctypes.data, q.ctypes.data, o.ctypes.data,
                        sh.ctypes.data, scene.sh_degree, 0 if self.feat is None else self.feat.shape[1],
                        None if self.feat is None else self.feat.ctypes.data,
                        *[self.ov[k].ctypes.data if k in self.ov else None
                          for k in ("means", "opacities", "log_scales", "quats", "sh", "feat")])
        self.c = _Camera(cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height, near,
                         (ctypes.c_double * 3)(*bg))


def _pose64(pose) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(12))


PROJ_FIELDS = ["u", "v", "z", "cov_xx", "cov_xy", "cov_yy", "conic_a", "conic_b", "conic_c", "o", "r", "g", "b",
               "rx", "ry", "mc_x", "mc_y", "mc_z", "cov3_xx", "cov3_xy", "cov3_xz", "cov3_yy", "cov3_yz",
               "cov3_zz", "bx0", "bx1", "by0", "by1", "err_u", "err_v", "err_z"]


def project(scene, pose, cam, near=0.2) -> dict:
    """Per-Gaussian FP64 projection: returns a dict of (N,) arrays named as in
    PROJ_FIELDS plus visible, px0, px1, py0, py1."""
    lib = _load()
    b = _Bound(scene, cam, near)
    n = scene.means.shape[0]
    dbl = np.zeros((n, 31), dtype=np.float64)
    ints = np.zeros((n, 5), dtype=np.int32)
    lib.orc_project(ctypes.byref(b.s), _ptr(_pose64(pose)), ctypes.byref(b.c), _ptr(dbl), _ptr(ints))
    out = {k: dbl[:, i].copy() for i, k in enumerate(PROJ_FIELDS)}
    for i, k in enumerate(["visible", "px0", "px1", "py0", "py1"]):
        out[k] = ints[:, i].copy()
    return out


def render(scene, pose, cam, mode: str = "tiled", tile: int = 16, margin: int = 1, near: float = 0.2,
           bg=(0.0, 0.0, 0.0), want_lists: bool = False, list_cap: int = 256, overrides=None) -> dict:
    """Render one pose in FP64.  Returns rgb (3,H,W), depth (H,W), alpha (H,W),
    feat (D,H,W) or None, T (H,W), nblend (H,W), fragile (H,W) bool, stats
    {visible, keys, tested, blended}, and lists (H*W, list_cap) when asked.
    overrides: optional float64 arrays replacing scene parameters (as in
    render_frozen)."""
    lib = _load()
    b = _Bound(scene, cam, near, bg, overrides)
    H, W, D = cam.height, cam.width, b.s.feat_dim
    rgb = np.zeros((3, H, W)); depth = np.zeros((H, W)); alpha = np.zeros((H, W))
    feat = np.zeros((D, H, W)) if D else None
    T = np.zeros((H, W)); nb = np.zeros((H, W), dtype=np.int32); frag = np.zeros((H, W), dtype=np.uint8)
    stats = np.zeros(4, dtype=np.int64)
    lists = np.full((H * W, list_cap), -1, dtype=np.int32) if want_lists else None
    rc = lib.orc_render(ctypes.byref(b.s), _ptr(_pose64(pose)), ctypes.byref(b.c), 0 if mode == "brute" else 1,
                        tile, margin, _ptr(rgb), _ptr(depth), _ptr(alpha), _ptr(feat), _ptr(T), _ptr(nb),
                        _ptr(frag), _ptr(stats), _ptr(lists), list_cap)
    if rc == 2:
        raise RuntimeError("oracle: per-pixel contributor list exceeded list_cap")
    return dict(rgb=rgb, depth=depth, alpha=alpha, feat=feat, T=T, nblend=nb, fragile=frag.astype(bool),
                stats=dict(visible=int(stats[0]), keys=int(stats[1]), tested=int(stats[2]), blended=int(stats[3])),
                lists=lists)


def render_frozen(scene, pose, cam, lists, counts, near=0.2, bg=(0.0, 0.0, 0.0), overrides=None) -> dict:
    """Re-render with the per-pixel blend lists of a reference render held
    fixed (no gate, no stop): the smooth branch used for finite differences.
    overrides: optional dict of float64 arrays replacing the scene's means,
    opacities, log_scales, quats, sh or feat (feat as values, not bf16 bits)."""
    lib = _load()
    b = _Bound(scene, cam, near, bg, overrides)
    H, W, D = cam.height, cam.width, b.s.feat_dim
    lists = np.ascontiguousarray(lists, dtype=np.int32)
    counts = np.ascontiguousarray(counts, dtype=np.int32).reshape(-1)
    rgb = np.zeros((3, H, W)); depth = np.zeros((H, W)); alpha = np.zeros((H, W))
    feat = np.zeros((D, H, W)) if D else None
    T = np.zeros((H, W))
    lib.orc_render_frozen(ctypes.byref(b.s), _ptr(_pose64(pose)), ctypes.byref(b.c), _ptr(lists), _ptr(counts),
                          lists.shape[1], _ptr(rgb), _ptr(depth), _ptr(alpha), _ptr(feat), _ptr(T))
    return dict(rgb=rgb, depth=depth, alpha=alpha, feat=feat, T=T)


def tile_lists(scene, pose, cam, tile: int = 16, edge_px: float = 1e-3, near: float = 0.2):
    """Per-tile Gaussian lists in (z, index) order: (offsets (ntiles+1,),
    ids (total,), edge (N,) bool)."""
    lib = _load()
    b = _Bound(scene, cam, near)
    ntiles = ((cam.width + tile - 1) // tile) * ((cam.height + tile - 1) // tile)
    offsets = np.zeros(ntiles + 1, dtype=np.int64)
    edge = np.zeros(scene.means.shape[0], dtype=np.uint8)
    total = np.zeros(1, dtype=np.int64)
    pose64 = _pose64(pose)
    lib.orc_tile_lists(ctypes.byref(b.s), _ptr(pose64), ctypes.byref(b.c), tile, edge_px, _ptr(offsets), None, 0,
                       _ptr(edge), _ptr(total))
    ids = np.zeros(max(1, int(total[0])), dtype=np.int32)
    lib.orc_tile_lists(ctypes.byref(b.s), _ptr(pose64), ctypes.byref(b.c), tile, edge_px, _ptr(offsets), _ptr(ids),
                       ids.shape[0], _ptr(edge), _ptr(total))
    return offsets, ids[: int(total[0])], edge.astype(bool)


def contrib(scene, pose, cam, tile: int = 16, near: float = 0.2):
    """Per-Gaussian render visibility of one pose: (contrib, robust, touched)
    boolean (N,) arrays -- blended at some pixel; blended at some non-fragile
    pixel; reached by the walk of some fragile pixel."""
    lib = _load()
    b = _Bound(scene, cam, near)
    n = scene.means.shape[0]
    c = np.zeros(n, dtype=np.uint8); r = np.zeros(n, dtype=np.uint8); t = np.zeros(n, dtype=np.uint8)
    lib.orc_contrib(ctypes.byref(b.s), _ptr(_pose64(pose)), ctypes.byref(b.c), tile, _ptr(c), _ptr(r), _ptr(t))
    return c.astype(bool), r.astype(bool), t.astype(bool)


def min_q_box(rows: np.ndarray) -> np.ndarray:
    """Smallest conic distance a dx^2 + 2 b dx dy + c dy^2 of rectangles to
    means: rows (n, 9) [a, b, c, u, v, x0, x1, y0, y1]."""
    lib = _load()
    r = np.zeros((len(rows), 10))
    r[:, :9] = rows
    out = np.zeros(len(rows))
    lib.orc_min_q_box(_ptr(r), len(rows), _ptr(out))
    return out


def sh_basis(degree: int, dirs: np.ndarray) -> np.ndarray:
    lib = _load()
    d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((d.shape[0], (degree + 1) ** 2))
    lib.orc_sh_basis(degree, _ptr(d), d.shape[0], _ptr(out))
    return out


def num_threads() -> int:
    return int(_load().orc_num_threads())
