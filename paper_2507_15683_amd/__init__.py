"""MI355X tile rasterizer of 3D Gaussian splats (RGB, depth, alpha, feature
maps) with its pose/parameter backward and batched multi-pose rendering.

Thin Python binding over libhgsr.so (include/hgsr.h): PyTorch provides device
memory and the stream; every step of the renderer runs in the library's HIP
kernels.  Importing this module does not touch the GPU; the library is loaded
on first use and its absence is an error (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import (SCHED_AUTO, SCHED_GRID, SCHED_POSE_MAJOR, SCHED_TILE_MAJOR, SORT_BUCKET, SORT_LSD,  # noqa: F401
                   HgsrError, check)

__all__ = ["GaussianScene", "Intrinsics", "Renderer", "render", "residual", "pose_adam", "HgsrError",
           "SORT_BUCKET", "SORT_LSD", "SCHED_GRID", "SCHED_POSE_MAJOR", "SCHED_TILE_MAJOR", "SCHED_AUTO"]


def _stream_ptr(stream: Optional[torch.cuda.Stream] = None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclasses.dataclass
class Intrinsics:
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    def c(self) -> _lib.Intrinsics:
        return _lib.Intrinsics(self.fx, self.fy, self.cx, self.cy, self.width, self.height)

    @staticmethod
    def of(cam) -> "Intrinsics":
        return Intrinsics(float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy), int(cam.width), int(cam.height))


@dataclasses.dataclass
class GaussianScene:
    """Device-resident Gaussian scene (structure of arrays).  feat holds
    bfloat16 values (the same bits as the generator's uint16 arrays)."""
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    opacities: torch.Tensor
    sh: torch.Tensor
    sh_degree: int
    feat: Optional[torch.Tensor] = None
    part_offsets: Optional[torch.Tensor] = None
    part_bounds: Optional[torch.Tensor] = None

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def feat_dim(self) -> int:
        return 0 if self.feat is None else int(self.feat.shape[1])

    @property
    def device(self) -> torch.device:
        return self.means.device

    order: Optional[np.ndarray] = None  # Gaussian i is input Gaussian order[i] (spatial layout), or None

    @staticmethod
    def from_numpy(s, device="cuda", spatial: bool = False) -> "GaussianScene":
        """Upload a synth-style host scene.  spatial=True stores it in Morton
        order (within partitions; hgsr_host_spatial_order) and keeps the
        permutation in `order`."""
        perm = None
        if spatial:
            s, perm = spatial_layout(s)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        feat = None
        if s.feat is not None:
            feat = torch.from_numpy(np.ascontiguousarray(s.feat).view(np.int16)).to(device).view(torch.bfloat16)
        sc = GaussianScene(t(s.means), t(s.log_scales), t(s.quats), t(s.opacities), t(s.sh), int(s.sh_degree), feat)
        sc.order = perm
        if getattr(s, "part_offsets", None) is not None:
            sc.part_offsets = t(s.part_offsets.astype(np.int64))
            sc.part_bounds = torch.empty((len(s.part_offsets) - 1, 6), dtype=torch.float32, device=device)
            g = sc.c()
            check(_lib.load().hgsr_partition_bounds(ctypes.byref(g), _ptr(sc.part_bounds), _stream_ptr()),
                  "hgsr_partition_bounds")
        return sc

    def c(self, partitions: bool = True) -> _lib.Gaussians:
        for name in ("means", "log_scales", "quats", "opacities", "sh"):
            x = getattr(self, name)
            if x.dtype != torch.float32 or not x.is_contiguous() or not x.is_cuda:
                raise ValueError(f"{name} must be a contiguous float32 device tensor")
        use_parts = partitions and self.part_offsets is not None
        return _lib.Gaussians(
            self.n, self.means.data_ptr(), self.log_scales.data_ptr(), self.quats.data_ptr(),
            self.opacities.data_ptr(), self.sh.data_ptr(), self.sh_degree, self.feat_dim,
            None if self.feat is None else self.feat.data_ptr(),
            (self.part_offsets.shape[0] - 1) if use_parts else 0,
            self.part_offsets.data_ptr() if use_parts else None,
            self.part_bounds.data_ptr() if use_parts else None)

    def validate(self):
        g = self.c()
        check(_lib.load().hgsr_validate(ctypes.byref(g), _stream_ptr()), "hgsr_validate")


def spatial_order(means: np.ndarray, part_offsets: Optional[np.ndarray] = None) -> np.ndarray:
    """Morton order of the Gaussians (within partitions), computed on the
    host by hgsr_host_spatial_order."""
    m = np.ascontiguousarray(means, dtype=np.float32)
    n = int(m.shape[0])
    perm = np.empty(n, dtype=np.int64)
    offs = None if part_offsets is None else np.ascontiguousarray(part_offsets, dtype=np.int64)
    check(_lib.load().hgsr_host_spatial_order(m.ctypes.data, n, None if offs is None else offs.ctypes.data,
                                              0 if offs is None else len(offs) - 1, perm.ctypes.data),
          "hgsr_host_spatial_order")
    return perm


def spatial_layout(s):
    """A host scene (synth-style dataclass of numpy arrays) reordered into
    Morton order within its partitions; returns (reordered scene, perm) with
    Gaussian i of the result = Gaussian perm[i] of the input."""
    perm = spatial_order(s.means, getattr(s, "part_offsets", None))
    return dataclasses.replace(s, means=s.means[perm], log_scales=s.log_scales[perm], quats=s.quats[perm],
                               opacities=s.opacities[perm], sh=s.sh[perm],
                               feat=None if s.feat is None else s.feat[perm]), perm


def _host_scene(s) -> tuple:
    """A hgsr_host_scene over a synth-style host scene (numpy arrays with
    part_offsets); returns (struct, arrays kept alive)."""
    arrs = [np.ascontiguousarray(getattr(s, f), dtype=np.float32) for f in ("means", "log_scales", "quats",
                                                                            "opacities", "sh")]
    feat = None if s.feat is None else np.ascontiguousarray(s.feat).view(np.uint16)
    offs = np.ascontiguousarray(s.part_offsets, dtype=np.int64)
    vp = lambda a: None if a is None else a.ctypes.data
    hs = _lib.HostScene(int(arrs[0].shape[0]), *[vp(a) for a in arrs], int(s.sh_degree),
                        0 if feat is None else int(feat.shape[1]), vp(feat), int(len(offs) - 1), vp(offs))
    return hs, (arrs, feat, offs)


def host_partition_bounds(s) -> np.ndarray:
    """Per partition (n_parts, 6) boxes of a host scene, computed on the host
    (hgsr_host_partition_bounds)."""
    hs, keep = _host_scene(s)
    out = np.empty((hs.n_parts, 6), dtype=np.float32)
    check(_lib.load().hgsr_host_partition_bounds(ctypes.byref(hs), out.ctypes.data), "hgsr_host_partition_bounds")
    return out


def partition_plan(bounds: np.ndarray, poses: np.ndarray, K: "Intrinsics", near: float = 0.2,
                   motion_margin: float = 0.0) -> np.ndarray:
    """(P, n_parts) uint8: 1 where a partition box may reach pose p's image
    (hgsr_partition_plan, host only)."""
    b = np.ascontiguousarray(bounds, dtype=np.float32)
    q = np.ascontiguousarray(np.asarray(poses, dtype=np.float32).reshape(-1, 12))
    out = np.zeros((q.shape[0], b.shape[0]), dtype=np.uint8)
    kc = K.c()
    check(_lib.load().hgsr_partition_plan(b.ctypes.data, b.shape[0], q.ctypes.data, q.shape[0], ctypes.byref(kc),
                                          near, motion_margin, out.ctypes.data), "hgsr_partition_plan")
    return out


class StreamedScene:
    """The device descriptor a PartitionCache hands out for one batch: usable
    wherever a GaussianScene is (render, backward, significance); valid until
    the cache's next prepare."""

    def __init__(self, g: "_lib.Gaussians", device):
        self._g = g
        self.n = int(g.n)
        self.sh_degree = int(g.sh_degree)
        self.feat_dim = int(g.feat_dim)
        self.device = device

    def c(self, partitions: bool = True) -> "_lib.Gaussians":
        return self._g


class PartitionCache:
    """Out-of-core partitioned scene: the whole scene in pinned host memory,
    `n_slots` partitions on the device at a time (hgsr_pcache_*)."""

    def __init__(self, host_scene, n_slots: int):
        self.lib = _lib.load()
        hs, keep = _host_scene(host_scene)
        h = ctypes.c_void_p()
        check(self.lib.hgsr_pcache_create(ctypes.byref(h), ctypes.byref(hs), n_slots), "hgsr_pcache_create")
        self.pc = h
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stats = {}

    def prepare(self, poses, K: "Intrinsics", near: float = 0.2, motion_margin: float = 0.0,
                ahead=None, stream=None) -> StreamedScene:
        """Make what `poses` may see resident (hgsr_pcache_prepare); `ahead`
        (upcoming poses, optional) have their partitions uploaded behind this
        batch, overlapping its renders."""
        q = np.ascontiguousarray(np.asarray(poses.cpu() if isinstance(poses, torch.Tensor) else poses,
                                            dtype=np.float32).reshape(-1, 12))
        n_render = q.shape[0]
        if ahead is not None and len(ahead):
            qa = np.asarray(ahead.cpu() if isinstance(ahead, torch.Tensor) else ahead, dtype=np.float32)
            q = np.ascontiguousarray(np.concatenate([q, qa.reshape(-1, 12)]))
        g = _lib.Gaussians()
        st = _lib.PcacheStats()
        kc = K.c()
        check(self.lib.hgsr_pcache_prepare(self.pc, q.ctypes.data, q.shape[0], n_render, ctypes.byref(kc), near,
                                           motion_margin,
                                           ctypes.byref(g), ctypes.byref(st), _stream_ptr(stream)),
              "hgsr_pcache_prepare")
        self.stats = st.as_dict()
        return StreamedScene(g, self.device)

    def evict_all(self):
        check(self.lib.hgsr_pcache_evict_all(self.pc), "hgsr_pcache_evict_all")

    def close(self):
        if getattr(self, "pc", None):
            self.lib.hgsr_pcache_destroy(self.pc)
            self.pc = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SlotPolicy:
    """The partition cache's slot policy on its own (host only, no GPU):
    step(need) with need[k] = 1 (rendered views may see partition k), 2 (only
    upcoming views may) or 0 returns the batch's counts and its upload list
    [(partition, slot, release batch or -1, ahead)]."""

    def __init__(self, n_parts: int, n_slots: int):
        self.lib = _lib.load()
        h = ctypes.c_void_p()
        check(self.lib.hgsr_slot_policy_create(ctypes.byref(h), n_parts, n_slots), "hgsr_slot_policy_create")
        self.h = h
        self.n_parts = n_parts

    def step(self, need) -> dict:
        nd = np.ascontiguousarray(np.asarray(need, dtype=np.uint8).reshape(self.n_parts))
        st = _lib.PcacheStats()
        check(self.lib.hgsr_slot_policy_step(self.h, nd.ctypes.data, ctypes.byref(st)), "hgsr_slot_policy_step")
        return st.as_dict()

    def evict_all(self):
        check(self.lib.hgsr_slot_policy_evict_all(self.h), "hgsr_slot_policy_evict_all")

    def close(self):
        if getattr(self, "h", None):
            self.lib.hgsr_slot_policy_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_SORTS = {"bucket": SORT_BUCKET, "lsd": SORT_LSD}
_SCHEDS = {"grid": SCHED_GRID, "pose": SCHED_POSE_MAJOR, "tile": SCHED_TILE_MAJOR, "auto": SCHED_AUTO}
_FEATS = {"auto": _lib.FEAT_AUTO, "valu": _lib.FEAT_VALU, "mfma": _lib.FEAT_MFMA}


class Renderer:
    """One library context: owns the renderer's workspace and the state the
    backward needs.  Not thread safe; one per stream."""

    def __init__(self, record_hint: int = 0, key_hint: int = 0):
        self.lib = _lib.load()
        h = ctypes.c_void_p()
        check(self.lib.hgsr_ctx_create(ctypes.byref(h), record_hint, key_hint), "hgsr_ctx_create")
        self.ctx = h
        self._keep = None

    def close(self):
        if self.ctx:
            self.lib.hgsr_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def opts(self, tile=16, sort="bucket", schedule="grid", bg=(0.0, 0.0, 0.0), near=0.2, feat_bf16=False,
             lds_sort_cap=0, feat_accum="auto") -> _lib.Opts:
        return _lib.Opts(tile, _SORTS[sort], _SCHEDS[schedule], (ctypes.c_float * 3)(*bg), near, int(feat_bf16),
                         lds_sort_cap, _FEATS[feat_accum])

    def reserve(self, P, width, height, tile, records_per_pose, keys, n_gaussians):
        check(self.lib.hgsr_reserve(self.ctx, P, width, height, tile, records_per_pose, keys, n_gaussians),
              "hgsr_reserve")

    def alloc_outputs(self, scene: GaussianScene, P: int, K: Intrinsics, feat_bf16=False):
        dev = scene.device
        H, W = K.height, K.width
        out = dict(rgb=torch.empty((P, 3, H, W), dtype=torch.float32, device=dev),
                   depth=torch.empty((P, H, W), dtype=torch.float32, device=dev),
                   alpha=torch.empty((P, H, W), dtype=torch.float32, device=dev), feat=None)
        if scene.feat_dim:
            out["feat"] = torch.empty((P, scene.feat_dim, H, W), dtype=torch.bfloat16 if feat_bf16 else torch.float32,
                                      device=dev)
        return out

    def render_into(self, scene: GaussianScene, poses: torch.Tensor, K: Intrinsics, out: dict, opts: _lib.Opts,
                    stream=None):
        """Enqueue one render (no synchronisation)."""
        if poses.dtype != torch.float32 or not poses.is_contiguous() or poses.shape[-1] != 12:
            raise ValueError("poses must be a contiguous float32 (P, 12) device tensor")
        P = poses.shape[0]
        g = scene.c()
        o = _lib.Outputs(_ptr(out["rgb"]), _ptr(out["depth"]), _ptr(out["alpha"]), _ptr(out["feat"]))
        kc = K.c()
        self._keep = (scene, poses, out)
        check(self.lib.hgsr_render(self.ctx, ctypes.byref(g), _ptr(poses), P, ctypes.byref(kc), ctypes.byref(opts),
                                   ctypes.byref(o), _stream_ptr(stream)), "hgsr_render")

    def check_overflow(self, stream=None) -> int:
        f = ctypes.c_int32(0)
        check(self.lib.hgsr_check_overflow(self.ctx, ctypes.byref(f), _stream_ptr(stream)), "hgsr_check_overflow")
        return int(f.value)

    def render(self, scene: GaussianScene, poses: torch.Tensor, K: Intrinsics, tile=16, sort="bucket",
               schedule="grid", bg=(0.0, 0.0, 0.0), near=0.2, feat_bf16=False, lds_sort_cap=0, feat_accum="auto",
               out=None, check_overflow=True, stream=None) -> dict:
        """Render P poses; returns dict(rgb (P,3,H,W), depth (P,H,W), alpha
        (P,H,W), feat (P,D,H,W) or None).  With check_overflow the call
        synchronises, and re-renders after growing the workspace if needed."""
        if poses.dim() == 1:
            poses = poses[None]
        P = poses.shape[0]
        if out is None:
            out = self.alloc_outputs(scene, P, K, feat_bf16)
        opts = self.opts(tile, sort, schedule, bg, near, feat_bf16, lds_sort_cap, feat_accum)
        for _ in range(6):
            self.render_into(scene, poses, K, out, opts, stream)
            if not check_overflow or self.check_overflow(stream) == 0:
                return out
        raise HgsrError(3, "render: workspace kept overflowing")

    def stats(self, stream=None) -> dict:
        s = _lib.RenderStats()
        check(self.lib.hgsr_stats(self.ctx, ctypes.byref(s), _stream_ptr(stream)), "hgsr_stats")
        return dict(visible=s.visible, keys=s.keys, max_tile_list=s.max_tile_list, overflow=s.overflow, tile=s.tile)

    def tile_lists(self, pose: int, n_tiles: int, cap: int, stream=None):
        """Per-tile Gaussian lists of the last render in blend order:
        (ranges (n_tiles, 2), gids)."""
        ranges = np.zeros((n_tiles, 2), dtype=np.uint32)
        gids = np.zeros(max(cap, 1), dtype=np.uint32)
        n = ctypes.c_int64(0)
        check(self.lib.hgsr_debug_tile_lists(self.ctx, pose, ranges.ctypes.data_as(ctypes.c_void_p),
                                             gids.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(n),
                                             _stream_ptr(stream)), "hgsr_debug_tile_lists")
        return ranges, gids[: n.value]

    @staticmethod
    def alloc_grads(scene: GaussianScene, P: int, want=("pose", "means", "opacities")) -> dict:
        dev = scene.device
        n, D, K = scene.n, scene.feat_dim, (scene.sh_degree + 1) ** 2
        shapes = dict(pose=(P, 6), means=(n, 3), opacities=(n,), log_scales=(n, 3), quats=(n, 4), sh=(n, K, 3),
                      feat=(n, D))
        return {k: torch.empty(shapes[k], dtype=torch.float32, device=dev) for k in want}

    def render_id(self) -> int:
        """Id of this context's last render (0: none, or a scoring pass
        came after it); hgsr_render_id."""
        v = ctypes.c_int64(0)
        check(self.lib.hgsr_render_id(self.ctx, ctypes.byref(v)), "hgsr_render_id")
        return int(v.value)

    def backward(self, grad_out: dict, want=("pose", "means", "opacities"), P: Optional[int] = None,
                 scene: Optional[GaussianScene] = None, grads: Optional[dict] = None, stream=None,
                 render_id: int = 0) -> dict:
        """Gradients of the last render given dL/d{rgb, depth, alpha, feat}
        (device FP32 tensors; missing keys mean zero).  `want` names the
        gradients to compute among pose, means, opacities, log_scales, quats,
        sh, feat; `grads` may supply preallocated outputs (required under
        graph capture).  A non-zero render_id makes the call fail unless that
        render is still the last one.  Returns the dict of device tensors."""
        scene = scene if scene is not None else self._keep[0]
        P = P if P is not None else self._keep[1].shape[0]
        if grads is None:
            grads = self.alloc_grads(scene, P, want)
        go = _lib.GradOutputs(*[_ptr(_f32(grad_out.get(k))) for k in ("rgb", "depth", "alpha", "feat")])
        gr = _lib.Grads(*[_ptr(grads.get(k)) for k in ("pose", "means", "opacities", "log_scales", "quats", "sh",
                                                      "feat")], render_id)
        self._keep_grad = (grad_out, grads)
        check(self.lib.hgsr_render_backward(self.ctx, ctypes.byref(go), ctypes.byref(gr), _stream_ptr(stream)),
              "hgsr_render_backward")
        return grads

    def residual_backward(self, rgb_target: torch.Tensor, feat_target: Optional[torch.Tensor] = None,
                          lam_f: float = 1.0, want=("pose",), loss: Optional[torch.Tensor] = None,
                          grads: Optional[dict] = None, P: Optional[int] = None,
                          scene: Optional[GaussianScene] = None, stream=None, render_id: int = 0):
        """Loss and gradients of the refinement residual of the last render
        against targets ((P,3,H,W)/(P,D,H,W), or a single (1,...) target
        shared by all poses), formed inside the blend backward.  The last
        render's rgb and (FP32 or bf16) feature outputs must be unchanged.
        Returns (loss (P,), grads dict)."""
        scene = scene if scene is not None else self._keep[0]
        P = P if P is not None else self._keep[1].shape[0]
        if grads is None:
            grads = self.alloc_grads(scene, P, want)
        if loss is None:
            loss = torch.empty(P, dtype=torch.float32, device=scene.device)
        shared = int(rgb_target.shape[0] == 1 and P > 1)
        if not shared and rgb_target.shape[0] != P:
            raise ValueError("targets must hold one image per pose or a single shared one")
        rt = _lib.ResidualTargets(_ptr(_f32(rgb_target)), _ptr(_f32(feat_target)), lam_f, shared)
        gr = _lib.Grads(*[_ptr(grads.get(k)) for k in ("pose", "means", "opacities", "log_scales", "quats", "sh",
                                                      "feat")], render_id)
        self._keep_grad = (rgb_target, feat_target, loss, grads)
        check(self.lib.hgsr_residual_backward(self.ctx, ctypes.byref(rt), _ptr(loss), ctypes.byref(gr),
                                              _stream_ptr(stream)), "hgsr_residual_backward")
        return loss, grads

    def significance_into(self, scene: GaussianScene, poses: torch.Tensor, K: Intrinsics, maps: torch.Tensor,
                          score_sum: torch.Tensor, vis_count: torch.Tensor, opts: _lib.Opts,
                          visible: Optional[torch.Tensor] = None, layout: str = "planar", stream=None):
        """Enqueue one batch of significance scoring (Sec. 3.2, Eq. 4-5): maps
        (P, D, Hf, Wf) planar or (P, Hf, Wf, D) interleaved float32; adds to
        score_sum (N,) float32 and vis_count (N,) int32; visible (P, N) uint8
        or None.  No synchronisation."""
        if poses.dtype != torch.float32 or not poses.is_contiguous() or poses.shape[-1] != 12:
            raise ValueError("poses must be a contiguous float32 (P, 12) device tensor")
        if maps.dtype != torch.float32 or not maps.is_contiguous() or maps.dim() != 4:
            raise ValueError("maps must be a contiguous float32 4-D device tensor")
        P = poses.shape[0]
        inter = layout == "interleaved"
        D = maps.shape[3] if inter else maps.shape[1]
        Hf, Wf = (maps.shape[1], maps.shape[2]) if inter else (maps.shape[2], maps.shape[3])
        if maps.shape[0] != P or D != scene.feat_dim:
            raise ValueError("maps must hold one D-channel map per pose, D = the scene's feature_dim")
        if score_sum.dtype != torch.float32 or vis_count.dtype != torch.int32:
            raise ValueError("score_sum must be float32 and vis_count int32")
        if visible is not None and (visible.dtype != torch.uint8 or visible.numel() != P * scene.n):
            raise ValueError("visible must be a (P, N) uint8 tensor")
        g = scene.c()
        kc = K.c()
        fm = _lib.FeatureMaps(_ptr(maps), Wf, Hf, _lib.MAP_INTERLEAVED if inter else _lib.MAP_PLANAR)
        self._keep = (scene, poses, maps)
        check(self.lib.hgsr_significance(self.ctx, ctypes.byref(g), _ptr(poses), P, ctypes.byref(kc),
                                         ctypes.byref(opts), ctypes.byref(fm), _ptr(score_sum), _ptr(vis_count),
                                         _ptr(visible), _stream_ptr(stream)), "hgsr_significance")

    def significance(self, scene: GaussianScene, poses: torch.Tensor, K: Intrinsics, maps: torch.Tensor,
                     score_sum: Optional[torch.Tensor] = None, vis_count: Optional[torch.Tensor] = None,
                     want_visible: bool = False, layout: str = "planar", tile=16, sort="bucket", near=0.2,
                     stream=None) -> dict:
        """Score the Gaussians against P views and return dict(score_sum,
        vis_count, score (Eq. 6), visible (P, N) uint8 or None).  Pass
        score_sum / vis_count to accumulate over batches of views.  The call
        synchronises; after a workspace overflow it restores the sums, grows
        the workspace and scores the batch again."""
        if poses.dim() == 1:
            poses = poses[None]
        dev = scene.device
        n = scene.n
        if score_sum is None:
            score_sum = torch.zeros(n, dtype=torch.float32, device=dev)
        if vis_count is None:
            vis_count = torch.zeros(n, dtype=torch.int32, device=dev)
        visible = torch.empty((poses.shape[0], n), dtype=torch.uint8, device=dev) if want_visible else None
        opts = self.opts(tile, sort, "grid", near=near)
        s0, c0 = score_sum.clone(), vis_count.clone()
        for _ in range(6):
            self.significance_into(scene, poses, K, maps, score_sum, vis_count, opts, visible, layout, stream)
            if self.check_overflow(stream) == 0:
                score = significance_final(score_sum, vis_count, stream=stream)
                return dict(score_sum=score_sum, vis_count=vis_count, score=score, visible=visible)
            score_sum.copy_(s0)
            vis_count.copy_(c0)
        raise HgsrError(3, "significance: workspace kept overflowing")

    def match(self, q_coarse: torch.Tensor, r_coarse: torch.Tensor, q_fine: Optional[torch.Tensor] = None,
              r_fine: Optional[torch.Tensor] = None, tau_coarse: float = 0.1, tau_fine: float = 0.1,
              out: Optional[dict] = None, stream=None) -> dict:
        """Coarse-to-fine probabilistic mutual matching (Sec. 3.4, Eq. 11) of
        query and rendered bf16 feature maps (D, Hc, Wc) and, optionally,
        (D, 8 Hc, 8 Wc).  Returns dict(n_coarse (1,) uint32 -- read it after
        synchronising --, coarse_query, coarse_render, coarse_p, fine_query,
        fine_render, fine_p) on the device (see hgsr_match_out)."""
        for t in (q_coarse, r_coarse, q_fine, r_fine):
            if t is not None and (t.dtype != torch.bfloat16 or not t.is_contiguous() or t.dim() != 3):
                raise ValueError("feature maps must be contiguous bfloat16 (D, H, W) device tensors")
        D, Hc, Wc = q_coarse.shape
        if r_coarse.shape != q_coarse.shape:
            raise ValueError("query and rendered coarse maps must have the same shape")
        if (q_fine is None) != (r_fine is None):
            raise ValueError("give both fine maps or neither")
        if q_fine is not None and (q_fine.shape != (D, 8 * Hc, 8 * Wc) or r_fine.shape != q_fine.shape):
            raise ValueError("fine maps must be (D, 8 Hc, 8 Wc)")
        dev = q_coarse.device
        N = Hc * Wc
        if out is None:
            out = dict(n_coarse=torch.zeros(1, dtype=torch.int32, device=dev),
                       coarse_query=torch.empty(N, dtype=torch.int32, device=dev),
                       coarse_render=torch.empty(N, dtype=torch.int32, device=dev),
                       coarse_p=torch.empty(N, dtype=torch.float32, device=dev),
                       fine_query=torch.empty(N * 64 if q_fine is not None else 0, dtype=torch.int32, device=dev),
                       fine_render=torch.empty(N * 64 if q_fine is not None else 0, dtype=torch.int32, device=dev),
                       fine_p=torch.empty(N * 64 if q_fine is not None else 0, dtype=torch.float32, device=dev))
        mm = _lib.MatchMaps(_ptr(q_coarse), _ptr(r_coarse), _ptr(q_fine), _ptr(r_fine), D, Wc, Hc)
        mo = _lib.MatchOut(*[_ptr(out[k]) for k in ("n_coarse", "coarse_query", "coarse_render", "coarse_p",
                                                     "fine_query", "fine_render", "fine_p")])
        self._keep_match = (q_coarse, r_coarse, q_fine, r_fine, out)
        check(self.lib.hgsr_match(self.ctx, ctypes.byref(mm), tau_coarse, tau_fine, ctypes.byref(mo),
                                  _stream_ptr(stream)), "hgsr_match")
        return out

    def pnp(self, p2d: torch.Tensor, x3d: torch.Tensor, K: Intrinsics, pose0: torch.Tensor, samples: torch.Tensor,
            tau: float = 2.0, gn_iters: int = 10, refine_iters: int = 10, want_hyps: bool = False,
            want_inliers: bool = True, stream=None) -> dict:
        """Pose from 2D-3D correspondences (Sec. 3.4, Eq. 10) by RANSAC over
        the given 3-point samples and truncated-quadratic refinement, on the
        device.  p2d (n, 2), x3d (n, 3), pose0 (12,) float32; samples
        (n_hyp, 3) int32.  Returns dict(pose (12,), best, counts (n_hyp,),
        n_inliers, inliers (n,) uint8 or None, hyp_poses or None)."""
        for t, shp in ((p2d, 2), (x3d, 3)):
            if t.dtype != torch.float32 or not t.is_contiguous() or t.dim() != 2 or t.shape[1] != shp:
                raise ValueError("p2d must be (n, 2) and x3d (n, 3) contiguous float32 device tensors")
        if p2d.shape[0] != x3d.shape[0]:
            raise ValueError("p2d and x3d must hold the same number of correspondences")
        if samples.dtype != torch.int32 or not samples.is_contiguous() or samples.dim() != 2 or samples.shape[1] != 3:
            raise ValueError("samples must be a contiguous (n_hyp, 3) int32 device tensor")
        dev = p2d.device
        n, H = p2d.shape[0], samples.shape[0]
        out = dict(pose=torch.empty(12, dtype=torch.float32, device=dev),
                   best=torch.empty(1, dtype=torch.int32, device=dev),
                   counts=torch.empty(H, dtype=torch.int32, device=dev),
                   n_inliers=torch.empty(1, dtype=torch.int32, device=dev),
                   inliers=torch.empty(n, dtype=torch.uint8, device=dev) if want_inliers else None,
                   hyp_poses=torch.empty((H, 12), dtype=torch.float32, device=dev) if want_hyps else None)
        pose0 = _f32(pose0).reshape(12).contiguous()
        pb = _lib.PnpProblem(_ptr(p2d), _ptr(x3d), n, _ptr(samples), H, tau, gn_iters, refine_iters)
        pr = _lib.PnpResult(*[_ptr(out[k]) for k in ("pose", "best", "counts", "hyp_poses", "inliers", "n_inliers")])
        kc = K.c()
        self._keep_pnp = (p2d, x3d, samples, pose0, out)
        check(self.lib.hgsr_pnp(self.ctx, ctypes.byref(pb), ctypes.byref(kc), _ptr(pose0), ctypes.byref(pr),
                                _stream_ptr(stream)), "hgsr_pnp")
        return out

    def autotune(self, scene: GaussianScene, poses: torch.Tensor, K: Intrinsics, out: dict, sort="bucket",
                 feat_bf16=False, with_backward: bool = False, cache_path: Optional[str] = None,
                 stream=None) -> dict:
        """Time tile sizes 8/16/32, the blend schedules and the feature
        accumulations on this input (with_backward: each render followed by
        the pose backward, the cost of a refinement step); the winner becomes
        this renderer's default for tile=0 / schedule="auto" /
        feat_accum="auto"."""
        g = scene.c()
        kc = K.c()
        opts = self.opts(16, sort, "grid", feat_bf16=feat_bf16)
        o = _lib.Outputs(_ptr(out["rgb"]), _ptr(out["depth"]), _ptr(out["alpha"]), _ptr(out["feat"]))
        res = _lib.TuneResult()
        check(self.lib.hgsr_autotune(self.ctx, ctypes.byref(g), _ptr(poses), poses.shape[0], ctypes.byref(kc),
                                     ctypes.byref(opts), ctypes.byref(o), int(with_backward),
                                     None if cache_path is None else cache_path.encode(), ctypes.byref(res),
                                     _stream_ptr(stream)), "hgsr_autotune")
        return dict(tile=res.tile, schedule={0: "grid", 1: "pose", 2: "tile"}[res.schedule],
                    feat_accum={1: "valu", 2: "mfma"}.get(res.feat_accum, "valu"), ms=res.ms,
                    proj_group=res.proj_group)

    def profile(self, enable: bool):
        check(self.lib.hgsr_profile_enable(self.ctx, int(enable)), "hgsr_profile_enable")

    def profile_read(self) -> dict:
        ms = (ctypes.c_double * 6)()
        calls = (ctypes.c_int64 * 6)()
        check(self.lib.hgsr_profile_read(self.ctx, ms, calls), "hgsr_profile_read")
        names = ["project", "bin_sort", "blend", "blend_bwd", "project_bwd", "score"]
        return {names[k]: (ms[k], calls[k]) for k in range(6)}

    # graph capture
    def graph_begin(self, stream):
        check(self.lib.hgsr_graph_begin(self.ctx, _stream_ptr(stream)), "hgsr_graph_begin")

    def graph_end(self):
        check(self.lib.hgsr_graph_end(self.ctx), "hgsr_graph_end")

    def graph_launch(self, replays: int, stream=None):
        check(self.lib.hgsr_graph_launch(self.ctx, replays, _stream_ptr(stream)), "hgsr_graph_launch")


def _f32(t):
    if t is None:
        return None
    if t.dtype != torch.float32 or not t.is_contiguous():
        t = t.float().contiguous()
    return t


def render(scene: GaussianScene, poses: torch.Tensor, K: Intrinsics, renderer: Optional[Renderer] = None, **kw):
    r = renderer if renderer is not None else Renderer()
    return r.render(scene, poses, K, **kw)


def render_grad(renderer: Renderer, scene: GaussianScene, poses: torch.Tensor, out: dict, grad_out: dict,
                want=("pose", "means", "opacities")) -> dict:
    """Backward of renderer's last render (which must be `out` of `poses`)."""
    return renderer.backward(grad_out, want=want, P=poses.shape[0], scene=scene)


def pose_retract(poses: torch.Tensor, xi: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
    """Exp(xi) T per pose (hgsr_pose_retract): poses (P, 12), xi (P, 6)."""
    poses, xi = _f32(poses), _f32(xi)
    if out is None:
        out = torch.empty_like(poses)
    check(_lib.load().hgsr_pose_retract(_ptr(poses), _ptr(xi), poses.shape[0], _ptr(out), _stream_ptr(stream)),
          "hgsr_pose_retract")
    return out


def pose_tangent_grad(xi: torch.Tensor, g: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
    """dL/dxi = J_l(xi)^T g (hgsr_pose_tangent_grad): the pose gradient at
    Exp(xi) T carried back to xi."""
    xi, g = _f32(xi), _f32(g)
    if out is None:
        out = torch.empty_like(g)
    check(_lib.load().hgsr_pose_tangent_grad(_ptr(xi), _ptr(g), xi.shape[0], _ptr(out), _stream_ptr(stream)),
          "hgsr_pose_tangent_grad")
    return out


class _RenderFn(torch.autograd.Function):
    """Differentiable render at the poses Exp(xi) T: gradients flow to the
    pose tangent xi and to the Gaussian means and opacities.  The backward
    is refused (HgsrError, STATE) when the renderer has rendered again since
    this forward."""

    @staticmethod
    def forward(ctx, xi, means, opacities, renderer, scene, poses, K, kw):
        ctx.set_materialize_grads(False)  # unused outputs pass None: no zero images
        eff = pose_retract(poses, xi.detach())
        out = renderer.render(scene, eff, K, **kw)
        ctx.renderer = renderer
        ctx.scene = scene
        ctx.render_id = renderer.render_id()
        ctx.P = poses.shape[0]
        ctx.has_feat = out["feat"] is not None
        ctx.needs = (xi.requires_grad, means.requires_grad, opacities.requires_grad)
        ctx.save_for_backward(xi)
        feat = out["feat"] if out["feat"] is not None else torch.empty(0, device=poses.device)
        return out["rgb"], out["depth"], out["alpha"], feat

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_alpha, g_feat):
        (xi,) = ctx.saved_tensors
        want = [k for k, need in zip(("pose", "means", "opacities"), ctx.needs) if need]
        go = dict(rgb=g_rgb, depth=g_depth, alpha=g_alpha, feat=g_feat if ctx.has_feat else None)
        grads = ctx.renderer.backward(go, want=want or ("pose",), P=ctx.P, scene=ctx.scene,
                                      render_id=ctx.render_id)
        g_xi = pose_tangent_grad(xi.detach(), grads["pose"]) if ctx.needs[0] else None
        return (g_xi, grads.get("means"), grads.get("opacities"), None, None, None, None, None)


def render_differentiable(renderer: Renderer, scene: GaussianScene, poses: torch.Tensor, K: Intrinsics,
                          xi: Optional[torch.Tensor] = None, **kw):
    """Autograd form: renders the poses Exp(xi) T and returns (rgb, depth,
    alpha, feat); d/d xi is carried through the left Jacobian of the
    retraction (at xi = 0 it is the pose gradient in the left-perturbation
    tangent (rho, phi)).  Gradients reach scene.means / scene.opacities when
    they require grad.  The returned maps are the renderer's; another render
    on the same renderer before .backward() makes the backward fail."""
    P = poses.shape[0]
    if xi is None:
        xi = torch.zeros((P, 6), dtype=torch.float32, device=poses.device, requires_grad=True)
    kw = dict(kw)
    kw.setdefault("check_overflow", True)
    return _RenderFn.apply(xi, scene.means, scene.opacities, renderer, scene, poses, K, kw)


def residual(rgb, feat, rgb_t, feat_t, lam_f=1.0, out=None, stream=None):
    """Per-pose refinement residual and its gradients (HIP kernel).  `out` may
    supply preallocated (loss, g_rgb, g_feat) (required under graph capture)."""
    lib = _lib.load()
    P, _, H, W = rgb.shape
    D = 0 if feat is None else feat.shape[1]
    if out is None:
        loss = torch.empty(P, dtype=torch.float32, device=rgb.device)
        g_rgb = torch.empty_like(rgb)
        g_feat = torch.empty((P, D, H, W), dtype=torch.float32, device=rgb.device) if D else None
    else:
        loss, g_rgb, g_feat = out
    check(lib.hgsr_residual(_ptr(rgb), _ptr(feat), int(feat is not None and feat.dtype == torch.bfloat16),
                            _ptr(rgb_t), _ptr(feat_t), P, H, W, D, lam_f, _ptr(loss), _ptr(g_rgb), _ptr(g_feat),
                            _stream_ptr(stream)), "hgsr_residual")
    return loss, g_rgb, g_feat


def significance_final(score_sum: torch.Tensor, vis_count: torch.Tensor, out: Optional[torch.Tensor] = None,
                       stream=None) -> torch.Tensor:
    """S(g_j) = score_sum / vis_count (Eq. 6), 0 where the count is 0."""
    if out is None:
        out = torch.empty_like(score_sum)
    check(_lib.load().hgsr_significance_final(_ptr(score_sum), _ptr(vis_count), score_sum.numel(), _ptr(out),
                                         _stream_ptr(stream)), "hgsr_significance_final")
    return out


def backproject(depth: torch.Tensor, pose: torch.Tensor, K: Intrinsics, pix: torch.Tensor,
                out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """World points (n, 3) of rendered pixels pix (n,) int32 (row-major in
    the (H, W) depth map) under the render pose (12,)."""
    H, W = depth.shape[-2:]
    n = pix.numel()
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=depth.device)
    pose = _f32(pose).reshape(12).contiguous()
    kc = K.c()
    check(_lib.load().hgsr_backproject(_ptr(_f32(depth)), W, H, _ptr(pose), ctypes.byref(kc), _ptr(pix), n,
                                       _ptr(out), _stream_ptr(stream)), "hgsr_backproject")
    return out


def pose_consistency(poses: torch.Tensor, tau_deg: float = 20.0, stream=None):
    """Algorithm 2 over consecutive dense results poses (n, 12): returns
    (reliable (1,) int32, max_angle (1,) float32) on the device."""
    poses = _f32(poses).contiguous()
    rel = torch.empty(1, dtype=torch.int32, device=poses.device)
    ang = torch.empty(1, dtype=torch.float32, device=poses.device)
    check(_lib.load().hgsr_pose_consistency(_ptr(poses), poses.shape[0], tau_deg, _ptr(rel), _ptr(ang),
                                            _stream_ptr(stream)), "hgsr_pose_consistency")
    return rel, ang


def pose_adam(poses, grad, m, v, step, lr_rho=1e-2, lr_phi=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    lib = _lib.load()
    check(lib.hgsr_pose_adam(_ptr(poses), _ptr(grad), _ptr(m), _ptr(v), _ptr(step), poses.shape[0], lr_rho, lr_phi,
                             b1, b2, eps, _stream_ptr(stream)), "hgsr_pose_adam")
