"""Coarse-to-fine probabilistic mutual matching -- FP64 oracle, TEST
INFRASTRUCTURE ONLY (the test suite, the smoke check and the benchmark's
CPU-baseline leg use it; the HIP library never does).

Sec. 3.4 matches the query's feature maps with the rendered ones, coarse
level first, then fine windows:

  M_ij   = cos(q_i, r_j): cosine similarity of query position i and rendered
           position j;
  Eq. 11   P = softmax_j(M / tau) (.) softmax_i(M / tau): the row-wise softmax
           times the column-wise softmax, element by element;
  MNN      (i, j) is a correspondence when j maximises row i of P and i
           maximises column j of P;
  fine     for every coarse correspondence (i, j), the w x w fine positions
           inside coarse cell i of the query and inside cell j of the render
           are matched the same way (w = H_f / H_c).

Readings (the paper is silent on them): both levels' maps are inputs
(bfloat16 feature vectors, D x H x W, planar), the fine maps w times the
coarse resolution; the cosine is a.b / (|a| |b| + 1e-8), as in the refinement
residual; argmax ties go to the lowest index; tau is a parameter per level;
fine correspondences are listed per coarse correspondence in the order of
the query's window positions (row-major), coarse ones in the order of the
query's positions.

An FP32 implementation reaches the same correspondences except where an
argmax is decided by less than its rounding: `margins` reports, per row and
column, the gap between the best and the second-best log-probability.
"""
from __future__ import annotations

import numpy as np

COS_EPS = 1e-8


def bf16_to_f64(bits: np.ndarray) -> np.ndarray:
    b = np.ascontiguousarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def vectors(fmap_bits: np.ndarray) -> np.ndarray:
    """(D, H, W) bf16 map -> (H * W, D) float64, positions row-major."""
    f = bf16_to_f64(fmap_bits)
    D = f.shape[0]
    return f.reshape(D, -1).T.copy()


def cosine_matrix(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    na = np.sqrt((A * A).sum(axis=1))
    nb = np.sqrt((B * B).sum(axis=1))
    return (A @ B.T) / (na[:, None] * nb[None, :] + COS_EPS)


def dual_softmax(M: np.ndarray, tau: float) -> np.ndarray:
    """Eq. 11: row softmax of M / tau times column softmax of M / tau."""
    S = M / tau
    er = np.exp(S - S.max(axis=1, keepdims=True))
    rows = er / er.sum(axis=1, keepdims=True)
    ec = np.exp(S - S.max(axis=0, keepdims=True))
    cols = ec / ec.sum(axis=0, keepdims=True)
    return rows * cols


def mnn(P: np.ndarray):
    """Mutual nearest neighbours of P: (i, j, P_ij) with j = argmax row i and
    i = argmax column j (lowest index on ties), ordered by i."""
    jr = np.argmax(P, axis=1)          # numpy: first maximum
    ic = np.argmax(P, axis=0)
    i = np.nonzero(ic[jr] == np.arange(P.shape[0]))[0]
    j = jr[i]
    return i, j, P[i, j]


def margins(P: np.ndarray):
    """Per row and per column: log of best / second-best probability (inf
    when there is one candidate)."""
    with np.errstate(divide="ignore"):
        L = np.log(P)
    def gap(X):
        if X.shape[1] < 2:
            return np.full(X.shape[0], np.inf)
        part = -np.partition(-X, 1, axis=1)[:, :2]
        with np.errstate(invalid="ignore"):
            g = part[:, 0] - part[:, 1]
        return np.where(np.isnan(g), 0.0, g)  # both underflowed to 0: a tie
    return gap(L), gap(L.T)


def coarse_matches(q_c: np.ndarray, r_c: np.ndarray, tau: float):
    """Coarse level: q_c, r_c (D, Hc, Wc) bf16 bits.  Returns dict(i, j, p,
    row_margin, col_margin, P)."""
    M = cosine_matrix(vectors(q_c), vectors(r_c))
    P = dual_softmax(M, tau)
    i, j, p = mnn(P)
    rm, cm = margins(P)
    return dict(i=i, j=j, p=p, row_margin=rm, col_margin=cm, P=P)


def window(cell: int, Wc: int, Wf: int, w: int) -> np.ndarray:
    """Fine positions (row-major) of coarse cell `cell`: w x w of them."""
    yc, xc = divmod(int(cell), Wc)
    ys = np.arange(w * yc, w * yc + w)
    xs = np.arange(w * xc, w * xc + w)
    return (ys[:, None] * Wf + xs[None, :]).reshape(-1)


def fine_matches(q_f: np.ndarray, r_f: np.ndarray, ci: np.ndarray, cj: np.ndarray, Wc: int, tau: float, w: int):
    """Fine level for coarse correspondences (ci, cj): per correspondence the
    w x w windows, Eq. 11 and MNN.  Returns dict(k, qi, rj, p, row_margin,
    col_margin): k the coarse correspondence, qi / rj fine positions (row-major
    in the fine maps), and per coarse correspondence the window's smallest
    row and column margins."""
    Wf = q_f.shape[2]
    qv, rv = vectors(q_f), vectors(r_f)
    ks, qs, rs, ps, rmin, cmin = [], [], [], [], [], []
    for k, (a, b) in enumerate(zip(ci, cj)):
        wq = window(a, Wc, Wf, w)
        wr = window(b, Wc, Wf, w)
        P = dual_softmax(cosine_matrix(qv[wq], rv[wr]), tau)
        i, j, p = mnn(P)
        rm, cm = margins(P)
        ks.append(np.full(len(i), k)); qs.append(wq[i]); rs.append(wr[j]); ps.append(p)
        rmin.append(rm.min()); cmin.append(cm.min())
    cat = lambda x, dt: np.concatenate(x).astype(dt) if x else np.zeros(0, dt)
    return dict(k=cat(ks, np.int64), qi=cat(qs, np.int64), rj=cat(rs, np.int64), p=cat(ps, np.float64),
                row_margin=np.asarray(rmin), col_margin=np.asarray(cmin))
