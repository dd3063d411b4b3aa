"""GPU forward parity: the HIP path (through the C ABI) against the FP64
oracle, element by element, plus bitwise self-consistency of the HIP path
across tile sizes, sort paths, launch schedules, batching and workspace
regrowth."""
import numpy as np
import pytest

import synth
from gpu_util import log, parity, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2507_15683_amd as hg
    return hg


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


def _poses(P):
    import torch
    return torch.from_numpy(np.ascontiguousarray(P, dtype=np.float32).reshape(-1, 12)).cuda()


def _render(hg, sc, P, cam, r=None, **kw):
    r = r or hg.Renderer()
    out = r.render(hg.GaussianScene.from_numpy(sc), _poses(P), hg.Intrinsics.of(cam), **kw)
    return out, r


def test_small_terrain_parity(hg, oracle_mod):
    log("case: terrain_20k_view k=0 tile16 bucket")
    sc, P, cam = synth.terrain_20k_view(0)
    out, r = _render(hg, sc, P, cam, tile=16)
    ref = oracle_mod.render(sc, P[0], cam, tile=16, margin=1)
    s = parity(out, ref, label="terrain_20k_view")
    st = r.stats()
    log("stats", st, "oracle", ref["stats"])
    assert st["visible"] >= ref["stats"]["visible"]


@pytest.mark.parametrize("seed", range(8))
def test_tiny_ragged_parity(hg, oracle_mod, seed):
    """Ragged image sizes, every tile size, both sort paths, SH degrees 0-3,
    feature widths 0/8/16/32/64."""
    n = 60 + 37 * seed
    D = [0, 8, 16, 32, 64, 32, 8, 16][seed]
    sc, P, cam = synth.tiny_scene(n, 100 + seed, width=67 + 5 * seed, height=45 + 3 * seed, sh_degree=seed % 4,
                                  feat_dim=D)
    ref = oracle_mod.render(sc, P[0], cam, tile=16, margin=1)
    for tile in (8, 16, 32):
        for sort in ("bucket", "lsd"):
            log(f"case: tiny seed={seed} n={n} D={D} tile={tile} sort={sort}")
            out, _ = _render(hg, sc, P, cam, tile=tile, sort=sort)
            parity(out, ref, label=f"tiny{seed}/t{tile}/{sort}", max_fragile_frac=0.05)


def compare_tile_lists(oracle_mod, r, sc, pose, cam, tile, label):
    """Every per-tile list of the renderer's last render (pose 0) against the
    oracle's exact listing: the same Gaussians apart from those whose tile set
    changes when a support-rectangle bound moves by 1e-3 px (edge-exempt,
    counted), no duplicates, and the oracle's (z, index) order apart from
    pairs whose FP64 depths lie within twice the sum of their FP32 depth
    error bounds (the renderer sorts FP32 depths; counted)."""
    off, ids, edge = oracle_mod.tile_lists(sc, pose, cam, tile=tile, edge_px=1e-3)
    proj = oracle_mod.project(sc, pose, cam)
    z, ez = proj["z"], proj["err_z"]
    ntiles = len(off) - 1
    ranges, gids = r.tile_lists(0, ntiles, cap=int(off[-1]) * 2 + 1024)
    assert int(ranges[-1, 1]) <= int(off[-1]) * 2 + 1024
    extra = missing = ties = worst = 0
    for t in range(ntiles):
        a = ids[off[t]:off[t + 1]].astype(np.int64)
        b = gids[ranges[t, 0]:ranges[t, 1]].astype(np.int64)
        assert len(np.unique(b)) == len(b), (label, t, "duplicate entries")
        sa, sb = set(a.tolist()), set(b.tolist())
        for i in sb - sa:
            assert edge[i], (label, t, "GPU lists", i)
            extra += 1
        for i in sa - sb:
            assert edge[i], (label, t, "GPU misses", i)
            missing += 1
        a2 = a[~edge[a]]
        b2 = b[~edge[b]]
        if len(b2) < 2 or np.array_equal(a2, b2):
            continue
        rank = np.empty(int(a2.max()) + 1, dtype=np.int64)
        rank[a2] = np.arange(len(a2))
        rb = rank[b2]
        inv = np.triu(rb[:, None] > rb[None, :], 1)   # (i before j on the GPU) but j first in the oracle
        ii, jj = np.nonzero(inv)
        dz = np.abs(z[b2[ii]] - z[b2[jj]])
        bound = 2.0 * (ez[b2[ii]] + ez[b2[jj]])
        assert np.all(dz <= bound), (label, t, b2[ii][dz > bound][:4], b2[jj][dz > bound][:4])
        ties += len(ii)
        worst = max(worst, float((dz / bound).max(initial=0)))
    log(f"{label}: {int(off[-1])} oracle entries, {int(ranges[-1, 1])} GPU entries; edge-exempt {extra} extra, "
        f"{missing} missing; {ties} depth near-tie swaps (largest |dz| / bound {worst:.2f})")
    return dict(extra=extra, missing=missing, ties=ties)


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_tile_lists_match_oracle(hg, oracle_mod, tile):
    log(f"case: terrain_20k_view tile lists, tile {tile}")
    sc, P, cam = synth.terrain_20k_view(0)
    out, r = _render(hg, sc, P, cam, tile=tile)
    compare_tile_lists(oracle_mod, r, sc, P[0], cam, tile, f"20k/t{tile}")


def test_tile_lists_1080p_1m(hg, oracle_mod):
    """Every tile list of the 1920x1080 view of the 1M-Gaussian scene
    (8,160 tiles at 16 px) against the oracle's exact listing."""
    sc, P, cam = synth.aerial_1m_1080p(0)
    log("case: aerial_1m_1080p tile lists, tile 16")
    out, r = _render(hg, sc, P, cam, tile=16)
    st = compare_tile_lists(oracle_mod, r, sc, P[0], cam, 16, "1080p/1M/t16")
    assert st["extra"] + st["missing"] <= 1e-3 * r.stats()["keys"]


def test_tile_size_invariance_bitwise(hg):
    sc, P, cam = synth.terrain_20k_view(1)
    outs = []
    for tile in (8, 16, 32):
        log(f"case: terrain_20k_view k=1 tile={tile}")
        o, _ = _render(hg, sc, P, cam, tile=tile)
        outs.append(o)
    for o in outs[1:]:
        for k in ("rgb", "depth", "alpha"):
            assert np.array_equal(to_np(outs[0][k]), to_np(o[k])), k


def test_sort_paths_and_schedules_bitwise(hg):
    sc, P, cam = synth.tiny_scene(300, 7, width=96, height=80, feat_dim=16, sh_degree=3)
    Ps = synth.perturb_poses(P[0], 5, 3, 1.0, 2.0)
    base, _ = _render(hg, sc, Ps, cam)
    for sort in ("bucket", "lsd"):
        for sched in ("grid", "pose", "tile"):
            for tile in (8, 16, 32):
                log(f"case: 5 poses sort={sort} sched={sched} tile={tile}")
                o, _ = _render(hg, sc, Ps, cam, sort=sort, schedule=sched, tile=tile)
                for k in ("rgb", "depth", "alpha", "feat"):
                    assert np.array_equal(to_np(base[k]), to_np(o[k])), (sort, sched, tile, k)


@pytest.mark.parametrize("tile", [8, 16])
def test_mfma_feature_accumulation(hg, oracle_mod, tile):
    """The matrix-core feature sum (32 channels) matches the oracle to the same
    bar, leaves colour/depth/alpha bitwise unchanged, and differs from the VALU
    sum only by association order."""
    sc, P, cam = synth.tiny_scene(500, 21, width=99, height=70, feat_dim=32, sh_degree=3)
    Ps = synth.perturb_poses(P[0], 3, 22, 1.0, 2.0)
    log(f"case: mfma features tile={tile}")
    mf, _ = _render(hg, sc, Ps, cam, tile=tile, feat_accum="mfma")
    va, _ = _render(hg, sc, Ps, cam, tile=tile, feat_accum="valu")
    for k in ("rgb", "depth", "alpha", "final_T"):
        if k in mf:
            assert np.array_equal(to_np(mf[k]), to_np(va[k])), k
    d = np.abs(to_np(mf["feat"]) - to_np(va["feat"])).max()
    log(f"mfma vs valu feature max abs diff {d:.3g}")
    assert d < 1e-5
    for p in range(len(Ps)):
        ref = oracle_mod.render(sc, Ps[p], cam, tile=16, margin=1)
        parity(mf, ref, p=p, label=f"mfma/t{tile}/{p}", max_fragile_frac=0.05)


def test_batched_equals_single(hg):
    sc, P, cam = synth.tiny_scene(400, 8, width=80, height=64, feat_dim=8, sh_degree=2)
    Ps = synth.perturb_poses(P[0], 7, 4, 1.5, 3.0)
    log("case: batched 7 poses vs single")
    batch, _ = _render(hg, sc, Ps, cam, schedule="tile")
    for p in range(len(Ps)):
        one, _ = _render(hg, sc, Ps[p:p + 1], cam)
        for k in ("rgb", "depth", "alpha", "feat"):
            assert np.array_equal(to_np(batch[k][p]), to_np(one[k][0])), (p, k)


def test_batched_equals_single_64_views_1m(hg):
    """The many-pose path (per-workgroup chunk box against each frustum,
    then per-Gaussian tests; chunked tile counting and emission) renders
    the 1M-Gaussian scene at 64 poses bit for bit as one-pose renders (the
    single-pass projection, which has no chunk test) do, at sampled poses."""
    sc, P, cam = synth.aerial_1m_64_views(0)
    sc, _ = hg.spatial_layout(sc)
    log("case: 64 poses at 960x540, 1M Gaussians, batched vs single at 6 poses")
    r = hg.Renderer()
    batch, _ = _render(hg, sc, P, cam, r=r, tile=16, feat_accum="valu")
    batch = {k: to_np(v) for k, v in batch.items() if v is not None}
    for p in (0, 7, 21, 38, 50, 63):
        one, _ = _render(hg, sc, P[p:p + 1], cam, tile=16, feat_accum="valu")
        for k in ("rgb", "depth", "alpha", "feat"):
            assert np.array_equal(batch[k][p], to_np(one[k][0])), (p, k)


def test_batched_equals_single_large_gaussians_at_borders(hg):
    """Large Gaussians close to the camera, with poses turned so that their
    supports straddle the image borders, where the chunk box test's margin
    is tightest: batched renders (chunk test) equal one-pose renders."""
    sc, P, cam = synth.tiny_scene(600, 77, width=96, height=72, feat_dim=8, sh_degree=1, altitude=12.0)
    sc = sc.copy()
    sc.log_scales[:] += np.log(6.0)
    Ps = synth.perturb_poses(P[0], 9, 78, 4.0, 25.0)
    log("case: large Gaussians at the borders, 9 poses batched vs single")
    batch, _ = _render(hg, sc, Ps, cam)
    seen = 0
    for p in range(len(Ps)):
        one, _ = _render(hg, sc, Ps[p:p + 1], cam)
        for k in ("rgb", "depth", "alpha", "feat"):
            assert np.array_equal(to_np(batch[k][p]), to_np(one[k][0])), (p, k)
        seen += int(to_np(one["alpha"][0]).max() > 0)
    assert seen > len(Ps) // 2


def test_more_than_64_poses(hg, oracle_mod):
    """Poses beyond one projection launch (64) go through further launches."""
    sc, P, cam = synth.tiny_scene(150, 9, width=40, height=32)
    Ps = synth.perturb_poses(P[0], 70, 5, 1.0, 2.0)
    log("case: 70 poses")
    out, _ = _render(hg, sc, Ps, cam, schedule="pose")
    for p in (0, 63, 64, 69):
        ref = oracle_mod.render(sc, Ps[p], cam)
        parity(out, ref, p=p, label=f"70poses/{p}", max_fragile_frac=0.05)


def test_empty_and_culled_scenes(hg):
    import torch
    sc, P, cam = synth.tiny_scene(50, 10)
    empty = sc.subset(np.zeros(0, dtype=np.int64))
    log("case: empty scene")
    out, _ = _render(hg, empty, P, cam, bg=(0.25, 0.5, 0.75))
    assert np.allclose(to_np(out["rgb"][0][1]), 0.5) and to_np(out["alpha"]).max() == 0
    behind = sc.copy()
    behind.means[:, 2] += 500.0  # everything above the camera: behind it
    log("case: all behind camera")
    out, _ = _render(hg, behind, P, cam)
    assert to_np(out["alpha"]).max() == 0 and to_np(out["depth"]).max() == 0
    faint = sc.copy()
    faint.opacities[:] = 0.5 / 255
    log("case: all below 1/255")
    out, _ = _render(hg, faint, P, cam)
    assert to_np(out["alpha"]).max() == 0


def _hand_scene(means, opac, rgb, sigma=1.0):
    """Camera-facing isotropic Gaussians of scale sigma with DC colours rgb."""
    n = len(means)
    sh = np.zeros((n, 1, 3), np.float32)
    sh[:, 0, :] = (np.asarray(rgb, np.float64) - 0.5) * (2.0 * np.sqrt(np.pi))
    return synth.Scene(np.asarray(means, np.float32), np.full((n, 3), np.log(sigma), np.float32),
                       np.tile(np.float32([1, 0, 0, 0]), (n, 1)), np.asarray(opac, np.float32), sh, 0, None)


def test_stop_clamps_and_ties_match_oracle(hg, oracle_mod):
    """Hand-built edge cases against the oracle: layers whose transmittance
    crosses the 1e-4 stop just after (7e-5: not blended) or just before
    (1.2e-4: blended) the fourth layer, an opaque Gaussian (alpha clamped at
    0.99), a negative SH colour (clamped at 0), and two Gaussians at one depth
    (taken in index order)."""
    cam = synth.Camera(100.0, 100.0, 32.5, 24.5, 64, 48)
    ident = np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]], np.float32)
    cols = np.random.default_rng(7).uniform(0, 1, (4, 3))
    cases = {f"stack o4={o4}": _hand_scene([[0, 0, 10 + k] for k in range(4)], [0.9] * 3 + [o4], cols)
             for o4 in (0.93, 0.88)}
    cases["opaque"] = _hand_scene([[0, 0, 10]], [1.0], [[0.2, 0.7, 0.4]])
    cases["negative colour"] = _hand_scene([[0, 0, 10]], [0.8], [[-0.4, 0.3, 1.2]])
    for name, sc in cases.items():
        log("case:", name)
        out, r = _render(hg, sc, ident, cam, tile=16)
        ref = oracle_mod.render(sc, ident[0], cam, tile=16, margin=1)
        parity(out, ref, label=name)
        assert to_np(out["alpha"][0])[24, 32] == pytest.approx(ref["alpha"][24, 32], abs=1e-6)
    # equal depths: index order, rgb = c0 a + c1 a (1 - a) at the common centre
    c = np.array([[1.0, 0.0, 0.2], [0.0, 1.0, 0.6]])
    for order in ([0, 1], [1, 0]):
        log("case: equal depths, order", order)
        sc = _hand_scene([[0, 0, 10]] * 2, [0.5, 0.5], c[order])
        out, _ = _render(hg, sc, ident, cam, tile=16)
        col = sc.sh[:, 0, :].astype(np.float64) / (2.0 * np.sqrt(np.pi)) + 0.5
        want = col[0] * 0.5 + col[1] * 0.25
        np.testing.assert_allclose(to_np(out["rgb"][0])[:, 24, 32], want, atol=1e-6)


def test_overflow_regrows_to_same_result(hg):
    sc, P, cam = synth.terrain_20k_view(2)
    log("case: default capacity")
    ref, _ = _render(hg, sc, P, cam)
    small = hg.Renderer(record_hint=1024, key_hint=2048)
    log("case: undersized workspace -> overflow -> regrow")
    opts = small.opts()
    outs = small.alloc_outputs(hg.GaussianScene.from_numpy(sc), 1, hg.Intrinsics.of(cam))
    small.render_into(hg.GaussianScene.from_numpy(sc), _poses(P), hg.Intrinsics.of(cam), outs, opts)
    assert small.check_overflow() != 0
    out, _ = _render(hg, sc, P, cam, r=small)
    assert small.check_overflow() == 0
    for k in ("rgb", "depth", "alpha"):
        assert np.array_equal(to_np(ref[k]), to_np(out[k])), k


def test_lds_sort_fallback_bitwise(hg):
    sc, P, cam = synth.tiny_scene(300, 11, width=64, height=48, feat_dim=8)
    log("case: LDS sort cap 4 (global-memory radix path)")
    a, _ = _render(hg, sc, P, cam)
    b, r = _render(hg, sc, P, cam, lds_sort_cap=4)
    assert r.stats()["max_tile_list"] > 4
    for k in ("rgb", "depth", "alpha", "feat"):
        assert np.array_equal(to_np(a[k]), to_np(b[k])), k


def test_repeat_renders_bitwise(hg):
    sc, P, cam = synth.terrain_20k_view(3)
    r = hg.Renderer()
    log("case: determinism")
    a, _ = _render(hg, sc, P, cam, r=r)
    a = {k: (None if v is None else v.clone()) for k, v in a.items()}
    b, _ = _render(hg, sc, P, cam, r=r)
    for k in ("rgb", "depth", "alpha"):
        assert np.array_equal(to_np(a[k]), to_np(b[k])), k


def test_1080p_1m_full_parity(hg, oracle_mod):
    """1M Gaussians (SH3, 32-d features), 1920x1080: every pixel against the
    oracle; bf16 feature output within bf16 rounding of the FP32 one."""
    sc, P, cam = synth.aerial_1m_1080p(0)
    log("case: aerial_1m_1080p 1080p fp32 features")
    out, r = _render(hg, sc, P, cam, tile=16)
    log("stats", r.stats())
    ref = oracle_mod.render(sc, P[0], cam, tile=16, margin=1)
    log("oracle stats", ref["stats"])
    parity(out, ref, label="aerial_1m_1080p")
    log("case: aerial_1m_1080p bf16 features")
    ob, _ = _render(hg, sc, P, cam, tile=16, feat_bf16=True)
    f32 = to_np(out["feat"][0])
    fb = to_np(ob["feat"][0])
    assert np.all(np.abs(fb - f32) <= np.abs(f32) * 2.0 ** -8 + 1e-30)


def test_partitioned_equals_unpartitioned(hg, oracle_mod):
    """Per-pose partition culling changes no output: a partitioned scene
    renders bitwise like the same Gaussians without partitions, for poses
    that see one, several or no partitions."""
    import copy
    sc = synth.partitioned_scene(16_000, 200.0, 7, cells_per_side=4, sh_degree=1, feat_dim=8, boxes_per_km2=800,
                                 per_box=20)
    flat = copy.copy(sc)
    flat.part_offsets = None
    cam = synth.Camera(160.0, 160.0, 64.0, 48.0, 128, 96)
    poses = np.stack([synth.down_pose((-75.0, -75.0), 40.0), synth.down_pose((0.0, 0.0), 80.0, (0.2, -0.1)),
                      synth.down_pose((60.0, -25.0), 50.0, (0.0, 0.3), 1.0),
                      synth.down_pose((5000.0, 5000.0), 80.0)])
    log("case: 4 poses, partitioned vs flat")
    a, r = _render(hg, sc, poses, cam, schedule="pose")
    b, _ = _render(hg, flat, poses, cam, schedule="pose")
    for k in ("rgb", "depth", "alpha", "feat"):
        assert np.array_equal(to_np(a[k]), to_np(b[k])), k
    assert to_np(a["alpha"][3]).max() == 0  # looks at nothing
    ref = oracle_mod.render(sc, poses[1], cam)
    parity(a, ref, p=1, label="partitioned/1", max_fragile_frac=0.05)


def test_autotune_choice_and_cache(hg, tmp_path):
    """The autotuner returns a valid choice, the renderer then uses it, and the
    result equals the fixed default configuration (features within the
    association-order difference of the matrix-core sum); a second tuner on
    the same shape reads the cache file instead of timing."""
    sc, P, cam = synth.tiny_scene(800, 31, width=96, height=72, feat_dim=32, sh_degree=2)
    Ps = synth.perturb_poses(P[0], 6, 32, 1.0, 2.0)
    scene = hg.GaussianScene.from_numpy(sc)
    K = hg.Intrinsics.of(cam)
    r = hg.Renderer()
    out = r.alloc_outputs(scene, len(Ps), K)
    cache = str(tmp_path / "tune.jsonl")
    log("case: autotune 6 poses")
    res = r.autotune(scene, _poses(Ps), K, out, cache_path=cache)
    log("tuned", res)
    assert res["tile"] in (8, 16, 32) and res["schedule"] in ("grid", "pose", "tile")
    assert res["feat_accum"] in ("valu", "mfma") and res["ms"] > 0
    tuned = r.render(scene, _poses(Ps), K, tile=0, schedule="auto")
    assert r.stats()["tile"] == res["tile"]
    base, _ = _render(hg, sc, Ps, cam, tile=16, feat_accum="valu")
    for k in ("rgb", "depth", "alpha"):
        assert np.array_equal(to_np(tuned[k]), to_np(base[k])), k
    assert np.abs(to_np(tuned["feat"]) - to_np(base["feat"])).max() < 1e-5
    r2 = hg.Renderer()
    res2 = r2.autotune(scene, _poses(Ps), K, out, cache_path=cache)
    assert (res2["tile"], res2["schedule"], res2["feat_accum"]) == (res["tile"], res["schedule"], res["feat_accum"])
    assert abs(res2["ms"] - res["ms"]) < 1e-4
    # tuned on the refinement step's cost (render + pose backward): its own
    # cache entry, and a time that includes the backward
    rb = hg.Renderer()
    resb = rb.autotune(scene, _poses(Ps), K, out, with_backward=True, cache_path=cache)
    log("tuned with backward", resb)
    assert resb["tile"] in (8, 16, 32) and resb["ms"] > res["ms"]
    rb2 = hg.Renderer()
    resb2 = rb2.autotune(scene, _poses(Ps), K, out, with_backward=True, cache_path=cache)
    assert (resb2["tile"], resb2["schedule"]) == (resb["tile"], resb["schedule"])
    assert abs(resb2["ms"] - resb["ms"]) < 1e-4
    # one pose: the projection's grouping is tuned too, cached, and changes
    # no output
    out1 = r.alloc_outputs(scene, 1, K)
    r1 = hg.Renderer()
    res1 = r1.autotune(scene, _poses(Ps[:1]), K, out1, cache_path=cache)
    log("tuned one pose", res1)
    assert res1["proj_group"] in (1, 4)
    one = r1.render(scene, _poses(Ps[:1]), K, tile=16, feat_accum="valu")
    for k in ("rgb", "depth", "alpha", "feat"):
        assert np.array_equal(to_np(one[k][0]), to_np(base[k][0])), k
    r1b = hg.Renderer()
    res1b = r1b.autotune(scene, _poses(Ps[:1]), K, out1, cache_path=cache)
    assert res1b["proj_group"] == res1["proj_group"] and abs(res1b["ms"] - res1["ms"]) < 1e-4
