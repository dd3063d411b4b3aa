"""ctypes declarations of the C ABI in include/hgsr.h (argument marshalling
only; every step of the renderer runs in libhgsr.so's HIP kernels)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhgsr.so")

HGSR_OK = 0
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "HIP", 3: "CAPACITY", 4: "UNSUPPORTED", 5: "STATE"}

SORT_BUCKET, SORT_LSD = 0, 1
SCHED_GRID, SCHED_POSE_MAJOR, SCHED_TILE_MAJOR, SCHED_AUTO = 0, 1, 2, -1
FEAT_AUTO, FEAT_VALU, FEAT_MFMA = 0, 1, 2

P_ = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
F32 = ctypes.c_float


class Gaussians(ctypes.Structure):
    _fields_ = [("n", I64), ("means", P_), ("log_scales", P_), ("quats", P_), ("opacities", P_), ("sh", P_),
                ("sh_degree", I32), ("feat_dim", I32), ("feat", P_), ("n_parts", I32), ("part_offsets", P_),
                ("part_bounds", P_)]


class Intrinsics(ctypes.Structure):
    _fields_ = [("fx", F32), ("fy", F32), ("cx", F32), ("cy", F32), ("width", I32), ("height", I32)]


class Opts(ctypes.Structure):
    _fields_ = [("tile", I32), ("sort_mode", I32), ("schedule", I32), ("bg", F32 * 3), ("near_z", F32),
                ("feat_out_bf16", I32), ("lds_sort_cap", I32), ("feat_accum", I32)]


class Outputs(ctypes.Structure):
    _fields_ = [("rgb", P_), ("depth", P_), ("alpha", P_), ("feat", P_)]


class GradOutputs(ctypes.Structure):
    _fields_ = [("rgb", P_), ("depth", P_), ("alpha", P_), ("feat", P_)]


class Grads(ctypes.Structure):
    _fields_ = [("pose", P_), ("means", P_), ("opacities", P_), ("log_scales", P_), ("quats", P_), ("sh", P_),
                ("feat", P_), ("render_id", I64)]


class RenderStats(ctypes.Structure):
    _fields_ = [("visible", I64), ("keys", I64), ("max_tile_list", I64), ("overflow", I32), ("tile", I32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("tile", I32), ("schedule", I32), ("feat_accum", I32), ("ms", F32), ("proj_group", I32)]


class ResidualTargets(ctypes.Structure):
    _fields_ = [("rgb_target", P_), ("feat_target", P_), ("lam_f", F32), ("shared_target", I32)]


class FeatureMaps(ctypes.Structure):
    _fields_ = [("maps", P_), ("width", I32), ("height", I32), ("layout", I32)]


MAP_PLANAR, MAP_INTERLEAVED = 0, 1


class MatchMaps(ctypes.Structure):
    _fields_ = [("query_coarse", P_), ("render_coarse", P_), ("query_fine", P_), ("render_fine", P_), ("D", I32),
                ("coarse_width", I32), ("coarse_height", I32)]


class MatchOut(ctypes.Structure):
    _fields_ = [("n_coarse", P_), ("coarse_query", P_), ("coarse_render", P_), ("coarse_p", P_),
                ("fine_query", P_), ("fine_render", P_), ("fine_p", P_)]

class PnpProblem(ctypes.Structure):
    _fields_ = [("p2d", P_), ("x3d", P_), ("n", I64), ("samples", P_), ("n_hyp", I32), ("tau", F32),
                ("gn_iters", I32), ("refine_iters", I32)]


class PnpResult(ctypes.Structure):
    _fields_ = [("pose", P_), ("best", P_), ("counts", P_), ("hyp_poses", P_), ("inliers", P_),
                ("n_inliers", P_)]


class HostScene(ctypes.Structure):
    _fields_ = [("n", I64), ("means", P_), ("log_scales", P_), ("quats", P_), ("opacities", P_), ("sh", P_),
                ("sh_degree", I32), ("feat_dim", I32), ("feat", P_), ("n_parts", I32), ("part_offsets", P_)]


MAX_SLOTS = 64


class SlotUpload(ctypes.Structure):
    _fields_ = [("part", I32), ("slot", I32), ("release", I64), ("ahead", I32), ("reserved", I32)]


class PcacheStats(ctypes.Structure):
    _fields_ = [("needed", I32), ("hits", I32), ("uploads", I32), ("evictions", I32), ("bytes_uploaded", I64),
                ("total_uploads", I64), ("total_bytes", I64), ("n_slots", I32), ("slot_capacity", I64),
                ("device_bytes", I64), ("prefetched", I32), ("upload", SlotUpload * MAX_SLOTS)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "upload"}
        d["upload_list"] = [(u.part, u.slot, u.release, u.ahead) for u in self.upload[: self.uploads]]
        return d


# (name, argtypes) for every entry point declared in include/hgsr.h
SIGNATURES = {
    "hgsr_ctx_create": [ctypes.POINTER(P_), I64, I64],
    "hgsr_ctx_destroy": [P_],
    "hgsr_reserve": [P_, I32, I32, I32, I32, I64, I64, I64],
    "hgsr_render": [P_, ctypes.POINTER(Gaussians), P_, I32, ctypes.POINTER(Intrinsics), ctypes.POINTER(Opts),
                    ctypes.POINTER(Outputs), P_],
    "hgsr_render_noalloc": [ctypes.POINTER(Gaussians), P_, I32, ctypes.POINTER(Intrinsics), ctypes.POINTER(Opts),
                            ctypes.POINTER(Outputs), I64, I64, P_, P_],
    "hgsr_render_backward": [P_, ctypes.POINTER(GradOutputs), ctypes.POINTER(Grads), P_],
    "hgsr_residual_backward": [P_, ctypes.POINTER(ResidualTargets), P_, ctypes.POINTER(Grads), P_],
    "hgsr_residual": [P_, P_, I32, P_, P_, I32, I32, I32, I32, F32, P_, P_, P_, P_],
    "hgsr_pose_adam": [P_, P_, P_, P_, P_, I32, F32, F32, F32, F32, F32, P_],
    "hgsr_render_id": [P_, ctypes.POINTER(I64)],
    "hgsr_pose_retract": [P_, P_, I32, P_, P_],
    "hgsr_pose_tangent_grad": [P_, P_, I32, P_, P_],
    "hgsr_significance": [P_, ctypes.POINTER(Gaussians), P_, I32, ctypes.POINTER(Intrinsics), ctypes.POINTER(Opts),
                          ctypes.POINTER(FeatureMaps), P_, P_, P_, P_],
    "hgsr_significance_final": [P_, P_, I64, P_, P_],
    "hgsr_match": [P_, ctypes.POINTER(MatchMaps), F32, F32, ctypes.POINTER(MatchOut), P_],
    "hgsr_pnp": [P_, ctypes.POINTER(PnpProblem), ctypes.POINTER(Intrinsics), P_, ctypes.POINTER(PnpResult), P_],
    "hgsr_backproject": [P_, I32, I32, P_, ctypes.POINTER(Intrinsics), P_, I64, P_, P_],
    "hgsr_pose_consistency": [P_, I32, F32, P_, P_, P_],
    "hgsr_partition_bounds": [ctypes.POINTER(Gaussians), P_, P_],
    "hgsr_pcache_create": [ctypes.POINTER(P_), ctypes.POINTER(HostScene), I32],
    "hgsr_pcache_destroy": [P_],
    "hgsr_pcache_prepare": [P_, P_, I32, I32, ctypes.POINTER(Intrinsics), F32, F32, ctypes.POINTER(Gaussians),
                            ctypes.POINTER(PcacheStats), P_],
    "hgsr_pcache_evict_all": [P_],
    "hgsr_host_partition_bounds": [ctypes.POINTER(HostScene), P_],
    "hgsr_partition_plan": [P_, I32, P_, I32, ctypes.POINTER(Intrinsics), F32, F32, P_],
    "hgsr_host_spatial_order": [P_, I64, P_, I32, P_],
    "hgsr_slot_policy_create": [ctypes.POINTER(P_), I32, I32],
    "hgsr_slot_policy_destroy": [P_],
    "hgsr_slot_policy_step": [P_, P_, ctypes.POINTER(PcacheStats)],
    "hgsr_slot_policy_evict_all": [P_],
    "hgsr_validate": [ctypes.POINTER(Gaussians), P_],
    "hgsr_graph_begin": [P_, P_],
    "hgsr_graph_end": [P_],
    "hgsr_graph_launch": [P_, I32, P_],
    "hgsr_check_overflow": [P_, ctypes.POINTER(I32), P_],
    "hgsr_stats": [P_, ctypes.POINTER(RenderStats), P_],
    "hgsr_debug_tile_lists": [P_, I32, P_, P_, I64, ctypes.POINTER(I64), P_],
    "hgsr_autotune": [P_, ctypes.POINTER(Gaussians), P_, I32, ctypes.POINTER(Intrinsics), ctypes.POINTER(Opts),
                      ctypes.POINTER(Outputs), I32, ctypes.c_char_p, ctypes.POINTER(TuneResult), P_],
    "hgsr_probe_valu_rate": [ctypes.POINTER(ctypes.c_double), P_],
    "hgsr_profile_enable": [P_, I32],
    "hgsr_profile_read": [P_, P_, P_],
    "hgsr_last_error": [],
    "hgsr_version": [],
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libhgsr.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2507_15683_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name in ("hgsr_last_error", "hgsr_version") else ctypes.c_int
    _lib = lib
    return lib


class HgsrError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = load().hgsr_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int, where: str):
    if status != HGSR_OK:
        raise HgsrError(status, where)
