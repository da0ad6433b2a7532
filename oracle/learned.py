"""CPU oracle for the binariser and the float-kNN ground truth -- TEST
INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may use
this module; the GPU library never imports it and it imports nothing from the
GPU library. Everything is plain numpy in float64, written from the
definitions, with no blocking or reordering beyond them.

What it computes
  * ``srp_encode``   -- the plain binariser: the paper maps real-valued
    features to Hamming space so that locality is preserved (Sec. 3.1); the
    plain stand-in is sign-of-random-projection: bit j of a code is 1 iff
    <x, w_j> > 0 (strictly; the reading taken for sgn(0), Eq. 2), packed in
    the code layout of the graph builder (bit j = bit j % 64 of word j // 64).
  * ``float_knn``    -- exact real-valued nearest neighbours (the brute-force
    ground truth of Sec. 4.2): row q = the first K of (||x_q - y_j||^2, j)
    over the base rows j (excluding one given index per query, its own row),
    ties to the smaller index; squared distances by direct differences.
  * ``recall_at``    -- Eq. 3: |B_ann(q) ∩ B_exact(q)| / N, averaged over q.
  * ``mlp_forward`` / ``mlp_backward`` -- the learned encoder (a reading:
    the paper uses learned hashing but gives no objective or network):
    Z1 = X W1 + b1, H1 = tanh Z1, Z2 = H1 W2 + b2, H = tanh Z2; code bit
    j = [Z2_j > 0]. W1 is [d][h1], W2 is [h1][bits] (input-major).
  * ``triplet_loss`` -- the training objective (a reading):
    with relaxed distances d(u, v) = (B - <h_u, h_v>) / 2 (the Hamming
    distance when h is +-1), for triplets (anchor a, positive p, negative n):
      L = mean_t softplus((d_ap - d_an + margin) / tau)
          + lam_q * mean_{rows, bits} (|h| - 1)^2
          + lam_b * sum_bits (mean_rows h)^2
    and its gradient with respect to H.
  * ``adam_step``    -- Adam (Kingma & Ba) with bias correction.

Parity pins: ``tests/test_oracle_learned.py`` (finite differences for the
gradients, closed forms for SRP, Adam and recall, a library route and a tiny
loop for the float kNN).
"""
from __future__ import annotations

import numpy as np

NO_IDX = 0xFFFFFFFF


def pack_code_bits(bits01: np.ndarray) -> np.ndarray:
    """[n][b] of 0/1 -> [n][b // 64] uint64, bit j = bit j % 64 of word j // 64."""
    bits01 = np.ascontiguousarray(bits01, dtype=np.uint8)
    n, b = bits01.shape
    out = np.zeros((n, b // 64), dtype=np.uint64)
    for j in range(b):
        out[:, j // 64] |= bits01[:, j].astype(np.uint64) << np.uint64(j % 64)
    return out


def srp_projections(x: np.ndarray, proj: np.ndarray) -> np.ndarray:
    return np.asarray(x, dtype=np.float64) @ np.asarray(proj, dtype=np.float64)


def srp_encode(x: np.ndarray, proj: np.ndarray) -> np.ndarray:
    """Codes [n][bits/64]: bit j = 1 iff <x, proj[:, j]> > 0 (float64)."""
    return pack_code_bits(srp_projections(x, proj) > 0)


def srp_margin(x: np.ndarray, proj: np.ndarray) -> np.ndarray:
    """|<x, w_j>| / (||x|| ||w_j||): how far each bit is from its sign flip."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(proj, dtype=np.float64)
    num = np.abs(x @ w)
    den = np.linalg.norm(x, axis=1)[:, None] * np.linalg.norm(w, axis=0)[None, :]
    return num / np.maximum(den, 1e-300)


def float_knn(queries: np.ndarray, base: np.ndarray, K: int, exclude=None):
    """Exact squared-L2 kNN by direct differences in float64.

    exclude: per-query base index to leave out (-1: none). Returns
    (idx uint32 [nq][K], dist float64 [nq][K]), padded with NO_IDX / inf."""
    q = np.asarray(queries, dtype=np.float64)
    y = np.asarray(base, dtype=np.float64)
    nq = q.shape[0]
    idx = np.full((nq, K), NO_IDX, dtype=np.uint32)
    dist = np.full((nq, K), np.inf, dtype=np.float64)
    for i in range(nq):
        d = ((y - q[i]) ** 2).sum(axis=1)
        cand = np.arange(y.shape[0])
        if exclude is not None and exclude[i] >= 0:
            cand = cand[cand != exclude[i]]
        order = np.lexsort((cand, d[cand]))[:K]
        idx[i, :order.size] = cand[order]
        dist[i, :order.size] = d[cand[order]]
    return idx, dist


def recall_at(approx_idx: np.ndarray, exact_idx: np.ndarray, N: int) -> float:
    """Eq. 3: mean over rows of |first N approx ∩ first N exact| / N."""
    a = np.asarray(approx_idx)[:, :N]
    e = np.asarray(exact_idx)[:, :N]
    hits = [len(set(a[r].tolist()) & set(e[r].tolist())) for r in range(a.shape[0])]
    return float(np.mean(hits)) / N


def mlp_forward(X, W1, b1, W2, b2):
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ W1 + b1
    H1 = np.tanh(Z1)
    Z2 = H1 @ W2 + b2
    H = np.tanh(Z2)
    return dict(X=X, Z1=Z1, H1=H1, Z2=Z2, H=H)


def mlp_backward(cache, dH, W2):
    """Gradients of a scalar loss with respect to W1, b1, W2, b2 given dL/dH."""
    H, H1, X = cache["H"], cache["H1"], cache["X"]
    dZ2 = dH * (1.0 - H * H)
    dW2 = H1.T @ dZ2
    db2 = dZ2.sum(axis=0)
    dH1 = dZ2 @ np.asarray(W2, dtype=np.float64).T
    dZ1 = dH1 * (1.0 - H1 * H1)
    dW1 = X.T @ dZ1
    db1 = dZ1.sum(axis=0)
    return dict(W1=dW1, b1=db1, W2=dW2, b2=db2)


LOSS_DEFAULTS = dict(margin=2.0, tau=4.0, lam_q=0.1, lam_b=0.01)


def softplus(z):
    return np.logaddexp(0.0, z)


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def triplet_loss(H, B: int, margin=2.0, tau=4.0, lam_q=0.1, lam_b=0.01):
    """H: [3T][B] rows (anchors, then positives, then negatives). Returns (L, dL/dH)."""
    H = np.asarray(H, dtype=np.float64)
    T = H.shape[0] // 3
    a, p, n = H[:T], H[T:2 * T], H[2 * T:3 * T]
    d_ap = (B - (a * p).sum(axis=1)) / 2.0
    d_an = (B - (a * n).sum(axis=1)) / 2.0
    z = (d_ap - d_an + margin) / tau
    L_trip = softplus(z).mean()
    g = sigmoid(z) / (tau * T)          # dL/dz_t
    # d(d_ap)/da = -p/2, d(d_ap)/dp = -a/2; d(d_an)/da = -n/2, d(d_an)/dn = -a/2
    dH = np.zeros_like(H)
    dH[:T] = g[:, None] * (-p / 2.0 + n / 2.0)
    dH[T:2 * T] = g[:, None] * (-a / 2.0)
    dH[2 * T:] = g[:, None] * (a / 2.0)
    R = H.shape[0]
    absH = np.abs(H)
    L_q = lam_q * ((absH - 1.0) ** 2).mean()
    dH += lam_q * 2.0 * (absH - 1.0) * np.sign(H) / (R * B)
    mu = H.mean(axis=0)
    L_b = lam_b * (mu ** 2).sum()
    dH += lam_b * 2.0 * mu[None, :] / R
    return L_trip + L_q + L_b, dH


def adam_step(param, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t = 1 for the first); returns (param, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return param - lr * mh / (np.sqrt(vh) + eps), m, v
