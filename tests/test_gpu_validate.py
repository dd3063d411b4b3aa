"""hgsr_validate on device data: a clean scene passes; NaN or Inf in any
parameter array (bfloat16 features included), opacities outside [0, 1] and a
zero quaternion are rejected with HGSR_ERR_INVALID_ARG; a call on a stream
that is being captured is refused with HGSR_ERR_STATE (it allocates and
synchronises)."""
import numpy as np
import pytest

import synth
from gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2507_15683_amd as hg
    return hg


def _scene(hg):
    sc, _, _ = synth.tiny_scene(300, 81, feat_dim=16, sh_degree=2)
    return hg.GaussianScene.from_numpy(sc)


CASES = [("means", (17, 1), float("nan")), ("means", (299, 2), float("inf")), ("log_scales", (5, 0), float("-inf")),
         ("quats", (40, 3), float("nan")), ("opacities", (3,), 1.5), ("opacities", (100,), -0.25),
         ("opacities", (7,), float("nan")), ("sh", (250, 4, 1), float("nan")), ("feat", (123, 15), float("inf")),
         ("feat", (0, 0), float("nan"))]


def test_clean_scene_passes(hg):
    log("case: validate clean scene")
    _scene(hg).validate()


@pytest.mark.parametrize("name,idx,val", CASES)
def test_bad_entries_rejected(hg, name, idx, val):
    import torch
    log(f"case: validate {name}{idx} = {val}")
    sc = _scene(hg)
    arr = getattr(sc, name)
    if name == "sh":
        arr = arr.view(sc.n, -1, 3)
    with torch.no_grad():
        arr[idx] = val
    with pytest.raises(hg.HgsrError, match="INVALID_ARG"):
        sc.validate()


def test_zero_quaternion_rejected(hg):
    import torch
    sc = _scene(hg)
    log("case: validate zero quaternion")
    with torch.no_grad():
        sc.quats[9] = 0.0
    with pytest.raises(hg.HgsrError, match="INVALID_ARG"):
        sc.validate()


def test_refused_while_capturing(hg):
    import torch
    sc = _scene(hg)
    r = hg.Renderer()
    s = torch.cuda.Stream()
    xi = torch.zeros((2, 6), device="cuda")
    poses = torch.zeros((2, 12), device="cuda")
    out = torch.empty_like(poses)
    torch.cuda.synchronize()
    log("case: validate during capture")
    with torch.cuda.stream(s):
        r.graph_begin(s)
        hg.pose_retract(poses, xi, out=out, stream=s)
        with pytest.raises(hg.HgsrError, match="STATE"):
            hg._lib.check(hg._lib.load().hgsr_validate(hg.ctypes.byref(sc.c()), hg._stream_ptr(s)), "hgsr_validate")
        r.graph_end()
    torch.cuda.synchronize()
    sc.validate()
