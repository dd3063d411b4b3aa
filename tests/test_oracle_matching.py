"""Pins of the oracle's probabilistic mutual matching (Sec. 3.4, Eq. 11)
against hand-computed values, scipy's log-sum-exp, invariances and
constructed maps whose correspondences are known.  CPU only."""
import math

import numpy as np
from scipy.special import logsumexp

import synth
from oracle import matching as mt


def _bits(x):
    return synth.f32_to_bf16_bits(np.asarray(x, dtype=np.float32))


def _map(vecs, H, W):
    """(H*W, D) row-major positions -> (D, H, W) bf16 bits."""
    v = np.asarray(vecs, dtype=np.float32)
    return _bits(v.T.reshape(v.shape[1], H, W))


def test_two_by_two_by_hand():
    """q = (e0, e1), r = (e0, e1): M = I (up to the 1e-8 in the cosine), so
    with tau = 0.5 each row and column softmax is (a, b) with
    a = e^2 / (e^2 + 1): P = diag(a^2) + offdiag(b^2); matches (0,0), (1,1)."""
    e = np.eye(2, 4)
    c = mt.coarse_matches(_map(e, 1, 2), _map(e, 1, 2), tau=0.5)
    a = math.exp(2.0) / (math.exp(2.0) + 1.0)
    b = 1.0 - a
    np.testing.assert_allclose(c["P"], [[a * a, b * b], [b * b, a * a]], rtol=1e-7)
    assert list(c["i"]) == [0, 1] and list(c["j"]) == [0, 1]
    # margins: log of best over second-best, log(a^2 / b^2) = 4 per row and column
    np.testing.assert_allclose(c["row_margin"], [4.0, 4.0], rtol=1e-6)
    np.testing.assert_allclose(c["col_margin"], [4.0, 4.0], rtol=1e-6)


def test_many_to_one_keeps_one_mutual_pair():
    """Two identical query vectors both prefer render 0; column 0 ties and
    keeps the lower index, so only (0, 0) is mutual; render 1 (orthogonal to
    both queries) is matched by nobody."""
    q = np.array([[1.0, 0, 0, 0], [1.0, 0, 0, 0], [0, 0, 1.0, 0]])
    r = np.array([[1.0, 0, 0, 0], [0, 1.0, 0, 0], [0, 0, 1.0, 0]])
    c = mt.coarse_matches(_map(q, 1, 3), _map(r, 1, 3), tau=0.1)
    assert list(zip(c["i"], c["j"])) == [(0, 0), (2, 2)]


def test_dual_softmax_in_log_domain():
    """P_ij = exp(2 S_ij - LSE_j S_ij - LSE_i S_ij) with S = M / tau (the
    product of the two softmaxes written with scipy's logsumexp), and P is
    unchanged when a constant is added to M."""
    rng = np.random.default_rng(3)
    M = rng.uniform(-1, 1, (7, 9))
    for tau in (0.05, 0.1, 1.0):
        S = M / tau
        want = np.exp(2 * S - logsumexp(S, axis=1, keepdims=True) - logsumexp(S, axis=0, keepdims=True))
        np.testing.assert_allclose(mt.dual_softmax(M, tau), want, rtol=1e-12)
        np.testing.assert_allclose(mt.dual_softmax(M + 0.37, tau), want, rtol=1e-9)
    # rows and columns of P are each bounded by the corresponding softmax
    P = mt.dual_softmax(M, 0.1)
    assert (P.sum(axis=1) <= 1 + 1e-12).all() and (P.sum(axis=0) <= 1 + 1e-12).all()


def test_low_temperature_keeps_mutual_argmax_of_cosine():
    """As tau -> 0, tau log P_ij -> 2 M_ij - max_j' M_ij' - max_i' M_i'j, which
    is 0 (its largest value) exactly at the mutual maxima of M: every mutual
    argmax pair of the cosine matrix is an MNN correspondence, with P near 1,
    and every other correspondence has a lower P."""
    rng = np.random.default_rng(5)
    q = rng.normal(0, 1, (40, 16))
    r = rng.normal(0, 1, (50, 16))
    qm, rm = _map(q, 5, 8), _map(r, 5, 10)
    M = mt.cosine_matrix(mt.vectors(qm), mt.vectors(rm))
    jr, ic = M.argmax(axis=1), M.argmax(axis=0)
    mutual = {(i, int(jr[i])) for i in range(40) if ic[jr[i]] == i}
    c = mt.coarse_matches(qm, rm, tau=1e-5)
    got = {(int(a), int(b)): p for a, b, p in zip(c["i"], c["j"], c["p"])}
    assert len(mutual) > 5 and mutual <= set(got)
    assert min(got[k] for k in mutual) > 0.99
    others = [p for k, p in got.items() if k not in mutual]
    assert not others or max(others) < min(got[k] for k in mutual)


def test_permutation_is_recovered():
    """A render map that is a permutation of the query's positions (distinct
    random vectors) is matched back exactly, with P near 1 at low tau."""
    rng = np.random.default_rng(7)
    Hc, Wc, D = 6, 9, 32
    q = rng.normal(0, 1, (Hc * Wc, D))
    perm = rng.permutation(Hc * Wc)
    r = q[perm]                      # render position k shows query position perm[k]
    c = mt.coarse_matches(_map(q, Hc, Wc), _map(r, Hc, Wc), tau=0.05)
    inv = np.argsort(perm)
    assert np.array_equal(c["i"], np.arange(Hc * Wc)) and np.array_equal(c["j"], inv[np.arange(Hc * Wc)])
    assert c["p"].min() > 0.9


def test_fine_windows_recover_a_one_cell_shift():
    """The render's fine map is the query's shifted left by one coarse cell
    (w = 8 fine pixels): every coarse match pairs query cell (x+1, y) with
    render cell (x, y), and inside each window every fine pixel finds the
    pixel 8 columns to its left."""
    rng = np.random.default_rng(11)
    w, Hc, Wc, D = 8, 3, 5, 16
    Hf, Wf = Hc * w, Wc * w
    qf = rng.normal(0, 1, (D, Hf, Wf)).astype(np.float32)
    rf = rng.normal(0, 1, (D, Hf, Wf)).astype(np.float32)
    rf[:, :, : Wf - w] = qf[:, :, w:]
    qc = qf.reshape(D, Hc, w, Wc, w).mean(axis=(2, 4))
    rc = rf.reshape(D, Hc, w, Wc, w).mean(axis=(2, 4))
    c = mt.coarse_matches(_bits(qc), _bits(rc), tau=0.1)
    shifted = [(y * Wc + x + 1, y * Wc + x) for y in range(Hc) for x in range(Wc - 1)]
    got = set(zip(c["i"].tolist(), c["j"].tolist()))
    assert set(shifted) <= got
    sel = np.array([k for k, (a, b) in enumerate(zip(c["i"], c["j"])) if (a, b) in set(shifted)])
    f = mt.fine_matches(_bits(qf), _bits(rf), c["i"][sel], c["j"][sel], Wc, tau=0.1, w=w)
    assert len(f["qi"]) == len(sel) * w * w
    qy, qx = np.divmod(f["qi"], Wf)
    ry, rx = np.divmod(f["rj"], Wf)
    assert np.array_equal(qy, ry) and np.array_equal(qx - w, rx)
    # listed per coarse match in the query window's row-major order
    assert np.array_equal(f["k"], np.repeat(np.arange(len(sel)), w * w))
    assert (np.diff(f["qi"].reshape(len(sel), w * w), axis=1) > 0).all()
