"""Pins of the learned-binariser oracle (CPU only): finite differences for every
gradient, closed forms for the sign-of-random-projection binariser, Adam and
recall (Eq. 3), a library route and a pure-Python loop for the float kNN, and
planted mistakes that the pins must catch."""
import numpy as np
import pytest

from oracle import learned as L
from paper_2102_04656_amd import datagen


def small_net(seed, d=8, h1=16, B=8):
    g = np.random.default_rng(seed)
    W1 = g.standard_normal((d, h1)) * 0.5
    b1 = g.standard_normal(h1) * 0.1
    W2 = g.standard_normal((h1, B)) * 0.5
    b2 = g.standard_normal(B) * 0.1
    X = g.standard_normal((15, d))  # 5 triplets: anchors, positives, negatives
    return X, dict(W1=W1, b1=b1, W2=W2, b2=b2)


def loss_of(X, P, B, fwd=L.mlp_forward, loss=L.triplet_loss):
    return loss(fwd(X, P["W1"], P["b1"], P["W2"], P["b2"])["H"], B)[0]


def grads_of(X, P, B, fwd=L.mlp_forward, bwd=L.mlp_backward, loss=L.triplet_loss):
    cache = fwd(X, P["W1"], P["b1"], P["W2"], P["b2"])
    _, dH = loss(cache["H"], B)
    return bwd(cache, dH, P["W2"])


def fd_check(X, P, B, **kw):
    """Max relative error of analytic vs central-difference gradients."""
    G = grads_of(X, P, B, **{k: v for k, v in kw.items() if k in ("fwd", "bwd", "loss")})
    worst = 0.0
    for name, val in P.items():
        flat = val.reshape(-1)
        for i in range(flat.size):
            old = flat[i]
            flat[i] = old + 1e-6
            lp = loss_of(X, P, B, **{k: v for k, v in kw.items() if k in ("fwd", "loss")})
            flat[i] = old - 1e-6
            lm = loss_of(X, P, B, **{k: v for k, v in kw.items() if k in ("fwd", "loss")})
            flat[i] = old
            num = (lp - lm) / 2e-6
            ana = G[name].reshape(-1)[i]
            worst = max(worst, abs(num - ana) / (1e-4 + abs(num) + abs(ana)))
    return worst


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mlp_and_loss_gradients_match_finite_differences(seed):
    X, P = small_net(seed)
    assert fd_check(X, P, 8) < 1e-5  # central differences in float64; mistakes give ~1


def test_loss_gradient_wrt_codes_matches_finite_differences():
    g = np.random.default_rng(3)
    H = np.tanh(g.standard_normal((12, 8)))
    _, dH = L.triplet_loss(H, 8)
    for i in range(H.shape[0]):
        for j in range(H.shape[1]):
            Hp, Hm = H.copy(), H.copy()
            Hp[i, j] += 1e-6
            Hm[i, j] -= 1e-6
            num = (L.triplet_loss(Hp, 8)[0] - L.triplet_loss(Hm, 8)[0]) / 2e-6
            assert abs(num - dH[i, j]) < 1e-6 * max(1.0, abs(num))


def test_loss_closed_form():
    # +-1 codes: relaxed distances are Hamming distances; quantisation term 0
    B = 8
    a = np.array([[1, 1, 1, 1, -1, -1, -1, -1]], dtype=float)
    p = a.copy()
    p[0, :2] *= -1                          # d_ap = 2
    n = -a                                  # d_an = 8
    H = np.concatenate([a, p, n])
    mu = H.mean(axis=0)
    want = np.logaddexp(0, (2 - 8 + 2.0) / 4.0) + 0.01 * (mu ** 2).sum()
    assert abs(L.triplet_loss(H, B)[0] - want) < 1e-12


def mutant_backward(kind):
    def bwd(cache, dH, W2):
        H, H1, X = cache["H"], cache["H1"], cache["X"]
        dZ2 = dH if kind == "no_tanh_grad" else dH * (1.0 - H * H)
        dW2 = H1.T @ dZ2
        db2 = dZ2.sum(axis=0)
        dH1 = dZ2 @ (W2 if kind == "untransposed" and W2.shape[0] == W2.shape[1] else W2.T)
        dZ1 = dH1 * (1.0 - H1 * H1)
        if kind == "wrong_sign":
            dZ1 = -dZ1
        dW1 = X.T @ dZ1
        db1 = dZ1.sum(axis=0) if kind != "bias_mean" else dZ1.mean(axis=0)
        return dict(W1=dW1, b1=db1, W2=dW2, b2=db2)
    return bwd


@pytest.mark.parametrize("kind", ["no_tanh_grad", "wrong_sign", "bias_mean", "untransposed"])
def test_finite_differences_catch_planted_mistakes(kind):
    X, P = small_net(5, d=8, h1=8, B=8)  # square W2 so the transposition mistake is expressible
    assert fd_check(X, P, 8, bwd=mutant_backward(kind)) > 1e-3


def test_srp_signed_axis_projection_closed_form():
    # projection columns +-e_pi(j): <x, w_j> = s_j x_pi(j) exactly
    g = np.random.default_rng(4)
    d = bits = 128
    perm = g.permutation(d)
    s = g.choice([-1.0, 1.0], size=bits)
    W = np.zeros((d, bits))
    W[perm, np.arange(bits)] = s
    x = g.standard_normal((50, d))
    want_bits = (s[None, :] * x[:, perm]) > 0
    assert np.array_equal(L.srp_encode(x, W), datagen.pack_bits(want_bits.astype(np.uint8)))
    # zero projection: strict sign gives bit 0
    assert not L.srp_encode(np.zeros((3, d)), W).any()


def test_srp_margin_is_cosine():
    g = np.random.default_rng(5)
    x = g.standard_normal((10, 16))
    W = g.standard_normal((16, 64))
    m = L.srp_margin(x, W)
    for i in range(10):
        for j in range(64):
            c = abs(x[i] @ W[:, j]) / (np.linalg.norm(x[i]) * np.linalg.norm(W[:, j]))
            assert abs(m[i, j] - c) < 1e-12


def test_float_knn_library_route_and_loop():
    from sklearn.neighbors import NearestNeighbors
    g = np.random.default_rng(6)
    base = g.standard_normal((400, 24))
    q = base[:40] + 0.01 * g.standard_normal((40, 24))
    idx, dist = L.float_knn(q, base, 10)
    nn = NearestNeighbors(n_neighbors=10, algorithm="brute").fit(base)
    d2, i2 = nn.kneighbors(q)
    assert np.array_equal(idx, i2.astype(np.uint32))
    assert np.allclose(dist, d2 ** 2, rtol=1e-9, atol=1e-9)
    # excluding each query's own row (queries = base rows)
    idx, dist = L.float_knn(base[:30], base, 5, exclude=np.arange(30))
    for i in range(30):
        d = [(float(((base[j] - base[i]) ** 2).sum()), j) for j in range(400) if j != i]
        d.sort()
        assert [j for _, j in d[:5]] == list(idx[i])


def test_float_knn_ties_and_padding():
    base = np.array([[0.0], [1.0], [-1.0], [2.0]])
    idx, dist = L.float_knn(np.array([[0.0]]), base, 6, exclude=np.array([0]))
    assert list(idx[0]) == [1, 2, 3, L.NO_IDX, L.NO_IDX, L.NO_IDX]  # tie 1 vs 2 -> smaller index
    assert list(dist[0][:3]) == [1.0, 1.0, 4.0] and np.isinf(dist[0][3:]).all()


def test_recall_closed_forms():
    e = np.array([[1, 2, 3, 4], [5, 6, 7, 8]])
    assert L.recall_at(e, e, 4) == 1.0
    assert L.recall_at(e + 100, e, 4) == 0.0
    a = np.array([[4, 3, 9, 9], [5, 0, 0, 8]])  # 2 of 4 and 2 of 4
    assert L.recall_at(a, e, 4) == 0.5
    assert L.recall_at(a, e, 2) == 0.25  # first two: {4,3}∩{1,2} = 0, {5,0}∩{5,6} = 1


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3])
    p, m, v = L.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), t=1, lr=0.1)
    # bias-corrected moments equal g and g^2: the step is lr * g / (|g| + eps)
    assert np.allclose(p, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)


# Adam beyond the first step. With beta1 = 1/2, beta2 = 3/4, lr = 1/10 and
# eps = 0 the moments and bias corrections are small fractions, worked by hand:
#   gradients 1, 0, -1:
#     t=1: m = 1/2,  v = 1/4,    m^ = 1,    v^ = 1      step -1/10
#     t=2: m = 1/4,  v = 3/16,   m^ = 1/3,  v^ = 3/7    step -(1/3)/sqrt(3/7)/10 = -sqrt(7/27)/10
#     t=3: m = -3/8, v = 25/64,  m^ = -3/7, v^ = 25/37  step +(3/7)/(5/sqrt(37))/10 = +3 sqrt(37)/350
#   a constant gradient 2: m^ = 2 and v^ = 4 at every t, so every step is -1/10.
#   gradients 2, -2, 4:
#     t=1: m = 1,    v = 1,      m^ = 2,    v^ = 4      step -1/10
#     t=2: m = -1/2, v = 7/4,    m^ = -2/3, v^ = 4      step +1/30
#     t=3: m = 7/4,  v = 85/16,  m^ = 2,    v^ = 340/37 step -(2/10) sqrt(37/340)
_ADAM_G = np.array([[1.0, 2.0, 2.0], [0.0, 2.0, -2.0], [-1.0, 2.0, 4.0]])
_ADAM_WANT = np.array([
    [-0.1, -0.1, -0.1],
    [-0.1 - np.sqrt(7 / 27) / 10, -0.2, -1 / 15],
    [-0.1 - np.sqrt(7 / 27) / 10 + 3 * np.sqrt(37) / 350, -0.3,
     -1 / 15 - 0.2 * np.sqrt(37 / 340)],
])


def _adam_pin(step):
    """Three steps of `step` against the hand-worked parameters, or a
    description of the first mismatch."""
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 4):
        p, m, v = step(p, _ADAM_G[t - 1], m, v, t=t, lr=0.1, beta1=0.5, beta2=0.75, eps=0.0)
        if not np.allclose(p, _ADAM_WANT[t - 1], rtol=1e-12, atol=1e-15):
            return f"t={t}: {p} != {_ADAM_WANT[t - 1]}"
    return None


def test_adam_three_steps_closed_form():
    assert _adam_pin(L.adam_step) is None


def _planted_adam(kind):
    def step(param, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        m = beta1 * m + (1.0 - beta1) * grad
        v = beta2 * v + (1.0 - beta2) * grad * grad
        tc = 1 if kind == "bias_frozen_t1" else t
        mh = m / (1.0 - beta1 ** tc)
        vh = v / (1.0 - (beta1 if kind == "beta1_in_v" else beta2) ** tc)
        if kind == "no_v_correction":
            vh = v
        return param - lr * mh / (np.sqrt(vh) + eps), m, v
    return step


@pytest.mark.parametrize("kind", ["bias_frozen_t1", "beta1_in_v", "no_v_correction"])
def test_adam_pin_catches_planted_mistakes(kind):
    assert _adam_pin(_planted_adam(kind)) is not None, f"planted mistake {kind} passed"


def test_adam_planted_copy_without_mistake_passes():
    assert _adam_pin(_planted_adam("none")) is None


def test_torch_recall_matches_oracle_recall():
    """The recall the experiment reports (torch, on whatever device the
    tensors live) equals the oracle's set definition of Eq. 3, including rows
    with repeated entries and entries beyond N."""
    import torch
    from paper_2102_04656_amd import learned_codes
    g = np.random.default_rng(11)
    exact = np.stack([g.permutation(200)[:64] for _ in range(300)]).astype(np.int64)
    approx = exact.copy()
    for r in range(300):  # replace a random part of each row, some with repeats
        k = g.integers(0, 65)
        pos = g.choice(64, size=k, replace=False)
        approx[r, pos] = g.integers(0, 200, size=k)
    approx[::7, 1] = approx[::7, 0]  # a repeated graph entry
    for N in (1, 10, 32, 64):
        want = L.recall_at(approx, exact, N)
        got = learned_codes.recall_at(torch.from_numpy(approx), torch.from_numpy(exact), N)
        assert abs(got - want) < 1e-12, (N, got, want)
