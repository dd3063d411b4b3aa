"""GPU coarse-to-fine probabilistic mutual matching (Sec. 3.4, Eq. 11)
through the C ABI against the FP64 oracle: coarse correspondences and their
probabilities, fine windows slot by slot, constructed maps with known
answers, ragged sizes and every feature width, and the 1080p-sized workload
(135 x 240 coarse positions) against a blockwise oracle."""
import numpy as np
import pytest

import synth
from gpu_util import log

pytestmark = pytest.mark.gpu

MARGIN = 1e-3     # log-probability gap below which FP32 may pick another argmax
P_RTOL = 1e-4


@pytest.fixture(scope="module")
def hg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2507_15683_amd as hg
    return hg


@pytest.fixture(scope="module")
def mt():
    from oracle import matching
    return matching


def _bf(bits):
    import torch
    return torch.from_numpy(np.ascontiguousarray(bits).view(np.int16)).cuda().view(torch.bfloat16)


def _gpu(hg, q_c, r_c, q_f=None, r_f=None, tau=0.1, tau_f=0.1):
    import torch
    r = hg.Renderer()
    out = r.match(_bf(q_c), _bf(r_c), None if q_f is None else _bf(q_f), None if r_f is None else _bf(r_f),
                  tau_coarse=tau, tau_fine=tau_f)
    torch.cuda.synchronize()
    K = int(out["n_coarse"].cpu().numpy().view(np.uint32)[0])
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["K"] = K
    return res


def _coarse_parity(g, c, label):
    """GPU coarse correspondences against the oracle's, except rows and
    columns whose argmax margin is below MARGIN."""
    K = g["K"]
    gi, gj, gp = g["coarse_query"][:K], g["coarse_render"][:K], g["coarse_p"][:K]
    assert (np.diff(gi) > 0).all(), "correspondences are listed in query order"
    shaky_r = c["row_margin"] < MARGIN
    shaky_c = c["col_margin"] < MARGIN
    want = {(int(i), int(j)): p for i, j, p in zip(c["i"], c["j"], c["p"]) if not shaky_r[i] and not shaky_c[j]}
    got = {(int(i), int(j)): p for i, j, p in zip(gi, gj, gp)}
    got_clean = {k: v for k, v in got.items() if not shaky_r[k[0]] and not shaky_c[k[1]]}
    log(label, "oracle", len(c["i"]), "gpu", K, "clean oracle", len(want), "clean gpu", len(got_clean),
        "shaky rows", int(shaky_r.sum()), "shaky cols", int(shaky_c.sum()))
    assert set(want) == set(got_clean), (label, sorted(set(want) ^ set(got_clean))[:8])
    for k, p in want.items():
        assert abs(got[k] - p) <= P_RTOL * p + 1e-7, (label, k, got[k], p)
    assert shaky_r.mean() < 0.05 and shaky_c.mean() < 0.05
    return got


@pytest.mark.parametrize("D,Hc,Wc", [(32, 12, 16), (8, 7, 9), (16, 5, 13), (64, 9, 11), (32, 1, 1), (32, 3, 50)])
def test_coarse_and_fine_parity(hg, mt, D, Hc, Wc):
    """Random maps (the render a shifted, noisy copy of the query) at ragged
    sizes; coarse correspondences exactly; fine windows slot by slot where
    the window's margins are clear."""
    log(f"case: matching D={D} coarse {Wc}x{Hc}")
    q_c, r_c, q_f, r_f = synth.matching_maps(D, Hc, Wc, seed=D * 100 + Hc, shift=(3, 5), noise=0.3)
    c = mt.coarse_matches(q_c, r_c, tau=0.1)
    g = _gpu(hg, q_c, r_c, q_f, r_f)
    got = _coarse_parity(g, c, f"coarse D{D} {Wc}x{Hc}")
    # fine: the oracle's windows for the GPU's correspondences
    K = g["K"]
    gi, gj = g["coarse_query"][:K], g["coarse_render"][:K]
    f = mt.fine_matches(q_f, r_f, gi, gj, Wc, tau=0.1, w=8)
    checked = 0
    for k in range(K):
        if f["row_margin"][k] < MARGIN or f["col_margin"][k] < MARGIN:
            continue
        sel = f["k"] == k
        want_q = dict(zip(f["qi"][sel].tolist(), zip(f["rj"][sel].tolist(), f["p"][sel].tolist())))
        slots = slice(64 * k, 64 * k + 64)
        gq, gr, gp = g["fine_query"][slots], g["fine_render"][slots], g["fine_p"][slots]
        got_q = {int(a): (int(b), float(p)) for a, b, p in zip(gq, gr, gp) if a >= 0}
        assert set(got_q) == set(want_q), (k, sorted(set(got_q) ^ set(want_q))[:6])
        for qpos, (rpos, p) in want_q.items():
            assert got_q[qpos][0] == rpos
            assert abs(got_q[qpos][1] - p) <= P_RTOL * p + 1e-7
        # invalid slots are -1, -1, 0
        assert ((gq >= 0) == (gr >= 0)).all() and (gp[gq < 0] == 0).all()
        checked += 1
    log("fine windows checked", checked, "of", K)
    assert checked >= 0.8 * K


def test_constructed_permutation_and_shift(hg):
    """Known answers on the GPU: a permuted render map is matched back
    exactly; a render shifted by one coarse cell gives the shifted coarse
    pairs and, inside each window, every pixel its twin 8 columns over."""
    rng = np.random.default_rng(7)
    Hc, Wc, D = 6, 9, 32
    q = rng.normal(0, 1, (Hc * Wc, D)).astype(np.float32)
    perm = rng.permutation(Hc * Wc)
    qm = synth.f32_to_bf16_bits(q.T.reshape(D, Hc, Wc))
    rm = synth.f32_to_bf16_bits(q[perm].T.reshape(D, Hc, Wc))
    g = _gpu(hg, qm, rm, tau=0.05)
    inv = np.argsort(perm)
    assert g["K"] == Hc * Wc
    assert np.array_equal(g["coarse_query"], np.arange(Hc * Wc)) and np.array_equal(g["coarse_render"], inv)
    # one-cell shift
    w, Hc, Wc, D = 8, 3, 5, 16
    Hf, Wf = Hc * w, Wc * w
    qf = rng.normal(0, 1, (D, Hf, Wf)).astype(np.float32)
    rf = rng.normal(0, 1, (D, Hf, Wf)).astype(np.float32)
    rf[:, :, : Wf - w] = qf[:, :, w:]
    qc = qf.reshape(D, Hc, w, Wc, w).mean(axis=(2, 4))
    rc = rf.reshape(D, Hc, w, Wc, w).mean(axis=(2, 4))
    b = synth.f32_to_bf16_bits
    g = _gpu(hg, b(qc), b(rc), b(qf), b(rf))
    pairs = list(zip(g["coarse_query"][: g["K"]].tolist(), g["coarse_render"][: g["K"]].tolist()))
    for k, (a, c) in enumerate(pairs):
        if a % Wc == 0 or (a - 1) != c:
            continue
        gq, gr = g["fine_query"][64 * k: 64 * k + 64], g["fine_render"][64 * k: 64 * k + 64]
        assert (gq >= 0).all()
        assert np.array_equal(gq // Wf, gr // Wf) and np.array_equal(gq % Wf - w, gr % Wf)
    assert sum(1 for a, c in pairs if a % Wc != 0 and a - 1 == c) == Hc * (Wc - 1)


def _oracle_coarse_blockwise(mt, q_c, r_c, tau, block=2048):
    """The oracle's coarse level for large N without the N x N matrix: the
    same definitions (cosine, Eq. 11's two softmaxes, MNN), evaluated in
    row blocks with the log-sum-exps accumulated in FP64."""
    from scipy.special import logsumexp
    Q, R = mt.vectors(q_c), mt.vectors(r_c)
    nq, nr = Q.shape[0], R.shape[0]
    nQ = np.sqrt((Q * Q).sum(1)); nR = np.sqrt((R * R).sum(1))
    a = np.empty(nq)
    b_parts = []
    for s in range(0, nq, block):
        S = (Q[s:s + block] @ R.T) / (nQ[s:s + block, None] * nR[None, :] + mt.COS_EPS) / tau
        a[s:s + block] = logsumexp(S, axis=1)
        b_parts.append(logsumexp(S, axis=0))
    b = logsumexp(np.stack(b_parts), axis=0)
    row_best = np.empty(nq, dtype=np.int64); row_gap = np.empty(nq)
    col_val = np.full(nr, -np.inf); col_best = np.zeros(nr, dtype=np.int64)
    col_second = np.full(nr, -np.inf)
    for s in range(0, nq, block):
        S = (Q[s:s + block] @ R.T) / (nQ[s:s + block, None] * nR[None, :] + mt.COS_EPS) / tau
        L = 2 * S - a[s:s + block, None] - b[None, :]          # log P
        row_best[s:s + block] = L.argmax(axis=1)
        top2 = -np.partition(-L, 1, axis=1)[:, :2]
        row_gap[s:s + block] = top2[:, 0] - top2[:, 1]
        bi = L.argmax(axis=0); bv = L[bi, np.arange(nr)]
        L2 = L.copy(); L2[bi, np.arange(nr)] = -np.inf
        sv = L2.max(axis=0)
        better = bv > col_val
        col_second = np.where(better, np.maximum(col_val, sv), np.maximum(col_second, bv))
        col_best = np.where(better, s + bi, col_best)
        col_val = np.where(better, bv, col_val)
    col_gap = col_val - col_second
    i = np.nonzero(col_best[row_best] == np.arange(nq))[0]
    j = row_best[i]
    p = np.exp(2 * ((Q[i] * R[j]).sum(1) / (nQ[i] * nR[j] + mt.COS_EPS)) / tau - a[i] - b[j])
    return dict(i=i, j=j, p=p, row_margin=row_gap, col_margin=col_gap)


def test_full_size_1080p(hg, mt):
    """135 x 240 coarse positions (1920 x 1080 at 1/8) with D = 32 and the
    1080 x 1920 fine maps: every coarse correspondence against the blockwise
    oracle, and 300 sampled fine windows."""
    log("case: matching 135x240 coarse, 1080x1920 fine, D 32")
    q_c, r_c, q_f, r_f = synth.matching_maps(32, 135, 240, seed=9000, shift=(11, -6), noise=0.3)
    g = _gpu(hg, q_c, r_c, q_f, r_f)
    c = _oracle_coarse_blockwise(mt, q_c, r_c, 0.1)
    _coarse_parity(g, c, "coarse 1080p")
    K = g["K"]
    pick = np.random.default_rng(1).choice(K, size=min(300, K), replace=False)
    gi, gj = g["coarse_query"][:K], g["coarse_render"][:K]
    f = mt.fine_matches(q_f, r_f, gi[pick], gj[pick], 240, tau=0.1, w=8)
    checked = 0
    for n, k in enumerate(pick):
        if f["row_margin"][n] < MARGIN or f["col_margin"][n] < MARGIN:
            continue
        sel = f["k"] == n
        want = dict(zip(f["qi"][sel].tolist(), f["rj"][sel].tolist()))
        gq, gr = g["fine_query"][64 * k: 64 * k + 64], g["fine_render"][64 * k: 64 * k + 64]
        got = {int(a): int(b) for a, b in zip(gq, gr) if a >= 0}
        assert got == want, (k, sorted(set(got.items()) ^ set(want.items()))[:6])
        checked += 1
    log("full size: coarse correspondences", K, "fine windows checked", checked)
    assert checked >= 200 and K > 10000
