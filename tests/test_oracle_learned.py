"""Pins of the learned-proposal oracle against closed forms, group structure,
finite differences, an autograd formulation, brute force and the special
cases that reduce it to the exhaustive search."""
import numpy as np
import pytest

import oracle
from oracle import learned as ol
from paper_1501_04140_amd import synth


def _identity_net():
    """W1 = [I; -I; 0], W2 = I, W3 = [I, -I, 0], zero biases: f(u) = relu(u) - relu(-u) = u."""
    p = {name: np.zeros(shape) for name, shape in ol.SHAPES}
    p["W1"][:64, :] = np.eye(64)
    p["W1"][64:128, :] = -np.eye(64)
    p["W2"][:, :] = np.eye(256)
    p["W3"][:, :64] = np.eye(64)
    p["W3"][:, 64:128] = -np.eye(64)
    return np.concatenate([p[name].ravel() for name, _ in ol.SHAPES])


def _dihedral(block):
    out = []
    for k in range(4):
        r = np.rot90(block, -k)  # k quarter turns clockwise
        out += [r, np.fliplr(r)]
    return out


def test_param_count():
    assert ol.N_PARAMS == 64 * 256 + 256 + 256 * 256 + 256 + 256 * 64 + 64 == 98880
    assert synth.mlp_init(0).size == ol.N_PARAMS


def test_isometries_form_the_dihedral_group():
    base = np.arange(64).reshape(8, 8)
    ours = {tuple(base.ravel()[p]) for p in ol.iso_perms()}
    ref = {tuple(b.ravel()) for b in _dihedral(base)}
    assert len(ours) == 8 and ours == ref


def test_identity_network_embeds_the_orbit_sum():
    rng = np.random.default_rng(0)
    X = ol.block_vectors(rng.integers(0, 256, size=(5, 64)))
    G, _ = ol.embed(_identity_net(), X)
    for q in range(5):
        S = sum(b for b in _dihedral(X[q].reshape(8, 8))).ravel()
        assert np.allclose(G[q], S / np.linalg.norm(S), atol=1e-12)


def test_embedding_is_isometry_invariant():
    theta = synth.mlp_init(3).astype(np.float64)
    rng = np.random.default_rng(1)
    X = ol.block_vectors(rng.integers(0, 256, size=(4, 64)))
    G, _ = ol.embed(theta, X)
    for t in range(8):
        Gt, _ = ol.embed(theta, X[:, ol.iso_perms()[t]])
        assert np.allclose(Gt, G, atol=1e-12)


def test_block_vectors_and_blocks():
    img = synth.power_law(64, beta=2.0, seed=2)
    v = ol.block_vectors(ol.range_blocks(img, [[0, 0], [8, 16]]))
    assert np.allclose(v.sum(axis=1), 0, atol=1e-12)
    assert np.allclose(np.linalg.norm(v, axis=1), 1)
    assert np.array_equal(ol.range_blocks(img, [[8, 16]])[0], img[8:16, 16:24].ravel())
    assert not ol.block_vectors(np.full((1, 64), 77)).any()
    gy, gx = oracle.domain_grid(64, 64, 8, 4)
    for j in (0, 5, gx + 3, gy * gx - 1):
        y, x = (j // gx) * 4, (j % gx) * 4
        assert np.array_equal(ol.domain_blocks(img, 4, [j])[0], oracle.decimate(img, y, x, 8).ravel())


def _tiny_problem(seed=0, nr=5, nd=7):
    rng = np.random.default_rng(seed)
    theta = synth.mlp_init(seed).astype(np.float64)
    theta += rng.normal(0, 0.05, size=theta.shape)  # non-zero biases too
    XR = ol.block_vectors(rng.integers(0, 256, size=(nr, 64)))
    XD = ol.block_vectors(rng.integers(0, 1021, size=(nd, 64)))
    labels = rng.integers(0, nd, size=nr)
    return theta, XR, XD, labels


def test_gradient_matches_central_differences():
    theta, XR, XD, labels = _tiny_problem()
    tau = 0.25
    _, g = ol.loss_and_grad(theta, XR, XD, labels, tau)
    rng = np.random.default_rng(9)
    # parameters with a visible gradient in every tensor
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in ol.SHAPES])
    picks = np.concatenate([rng.choice(np.arange(offs[i], offs[i + 1]), 6, replace=False)
                            for i in range(len(ol.SHAPES))])
    h = 1e-6
    for i in picks:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (ol.loss_and_grad(tp, XR, XD, labels, tau)[0] -
              ol.loss_and_grad(tm, XR, XD, labels, tau)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])


def test_gradient_matches_autograd():
    torch = pytest.importorskip("torch")
    theta, XR, XD, labels = _tiny_problem(seed=4, nr=6, nd=9)
    tau = 0.1
    loss, g = ol.loss_and_grad(theta, XR, XD, labels, tau)
    t = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    parts, o = [], 0
    for _, shape in ol.SHAPES:
        size = int(np.prod(shape))
        parts.append(t[o:o + size].reshape(shape))
        o += size
    W1, b1, W2, b2, W3, b3 = parts

    def g_of(X):
        blocks = torch.tensor(X, dtype=torch.float64).reshape(-1, 8, 8)
        S = 0
        for k in range(4):
            r = torch.rot90(blocks, -k, dims=(1, 2))
            for b in (r, torch.flip(r, dims=(2,))):
                u = b.reshape(-1, 64)
                y = torch.relu(torch.relu(u @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
                S = S + y
        return S / S.norm(dim=1, keepdim=True)

    Z = g_of(XR) @ g_of(XD).T / tau
    L = torch.nn.functional.cross_entropy(Z, torch.tensor(labels))
    L.backward()
    assert abs(L.item() - loss) < 1e-12
    assert np.allclose(t.grad.numpy(), g, rtol=1e-9, atol=1e-12)


def test_uniform_logits_give_log_of_domain_count():
    theta, XR, _, _ = _tiny_problem(seed=2)
    XD = np.repeat(XR[:1], 11, axis=0)  # every domain embeds to the same vector
    loss, _ = ol.loss_and_grad(theta, XR, XD, np.arange(5) % 11, 0.5)
    assert abs(loss - np.log(11)) < 1e-12


def test_adam_constant_gradient_closed_form():
    g = synth.grad_like(1000, seed=1).astype(np.float64)
    theta = np.zeros(1000)
    m = np.zeros(1000)
    v = np.zeros(1000)
    lr, eps = 1e-3, 1e-8
    for step in range(1, 4):
        theta, m, v = ol.adam_step(theta, g, m, v, step, lr, eps=eps)
        # with a constant gradient the bias-corrected moments are g and g^2
        assert np.allclose(theta, -step * lr * g / (np.abs(g) + eps), rtol=1e-10, atol=1e-15)


def _codes_and_rows(n, seed, n_dup=0):
    """int8 codes with 127 in row 0 and their rows q * 2^-8 (exact in fp16), so that
    the common scale is 127 / (127 * 2^-8) = 256 and the codes come back unchanged."""
    rng = np.random.default_rng(seed)
    q = rng.integers(-127, 128, size=(n, 64))
    q[0, 0] = 127
    for i in range(1, n_dup + 1):
        q[-i] = q[i]
    return q, (q * 2.0 ** -8).astype(np.float16)


def test_quantize_recovers_exact_codes():
    qr, xr = _codes_and_rows(9, seed=1)
    qd, _ = _codes_and_rows(40, seed=2)
    qd = np.clip(qd, -100, 100)  # the scale is common: the domains' own largest value is 100
    xd = (qd * 2.0 ** -8).astype(np.float16)
    (cr, cd), s = ol.quantize(xr, xd)
    assert s == np.float32(256.0)
    assert np.array_equal(cr, qr) and np.array_equal(cd, qd)


def test_quantize_rounds_half_to_even():
    # scale 256: x = (2j + 1) 2^-9 lands on j + 1/2
    x = np.zeros((2, 64), np.float16)
    x[0, 0] = 127 * 2.0 ** -8
    x[1, :6] = np.array([1, 3, 5, -1, -3, -5]) * 2.0 ** -9
    (c,), _ = ol.quantize(x)
    assert list(c[1, :6]) == [0, 2, 2, 0, -2, -2]


def test_topk_brute_force_with_ties():
    qr, xr = _codes_and_rows(6, seed=3)
    qd, xd = _codes_and_rows(40, seed=4, n_dup=8)
    qd[5] = qd[30] = qr[0] * (qr[0] != 127)  # an exact tie at the top for range 0 ...
    qd[5, 0] = qd[30, 0] = 127               # ... keeping 127 as the largest code
    xd = (qd * 2.0 ** -8).astype(np.float16)
    got = ol.topk(xr, xd, 7)
    for q in range(6):
        scores = [(-sum(int(a) * int(b) for a, b in zip(qr[q], qd[j])), j) for j in range(40)]
        ref = [j for _, j in sorted(scores)[:7]]
        assert list(got[q]) == ref
    assert got[0][0] == 5 and got[0][1] == 30


def test_topk_equals_exact_ranking_where_separated():
    """Where the exact (fp64) similarities of the k-th and the (k+1)-th domain differ by
    more than twice the quantization error bound, the int8 proposals are the exact top-k."""
    GR = synth.unit_rows_f16(300, seed=5).astype(np.float64)
    GD = synth.unit_rows_f16(30, seed=6).astype(np.float64)
    k = 2
    (_, _), s = ol.quantize(GR, GD)
    s = float(s)
    got = ol.topk(GR, GD, k)
    S = GR @ GD.T
    checked = 0
    for q in range(300):
        # |q_r . q_d / s^2 - x_r . x_d| <= (|x_r|_1 + max |x_d|_1) / (2 s) + 64 / (4 s^2)
        bound = (np.abs(GR[q]).sum() + np.abs(GD).sum(1).max()) / (2 * s) + 16 / s ** 2
        order = np.argsort(-S[q], kind="stable")
        if S[q, order[k - 1]] - S[q, order[k]] > 2 * bound:
            assert set(got[q]) == set(order[:k].tolist())
            checked += 1
    assert checked >= 20


@pytest.fixture(scope="module")
def small_img():
    return synth.power_law(48, beta=2.0, seed=5)


def test_learned_match_with_every_domain_is_exhaustive(small_img):
    theta = synth.mlp_init(1)
    gy, gx = oracle.domain_grid(48, 48, 8, 4)
    m, fb, props = ol.learned_match(small_img, theta, 4, gy * gx, rms=1e9)
    ref = oracle.match_level(small_img, 8, 4)
    assert not fb.any() and props.shape == (36, gy * gx)
    for f in ("e_lit", "dom", "iso", "s_idx", "q_o"):
        assert np.array_equal(m[f], ref[f]), f


def test_learned_match_always_falling_back_is_exhaustive(small_img):
    m, fb, _ = ol.learned_match(small_img, synth.mlp_init(1), 4, 3, rms=0.0)
    ref = oracle.match_level(small_img, 8, 4)
    assert fb[ref["e_lit"] > 0].all()
    for f in ("e_lit", "dom", "iso", "s_idx"):
        assert np.array_equal(m[f], ref[f]), f


def test_learned_match_is_the_argmin_over_its_proposals(small_img):
    """Brute force over proposals x isometries x s with the literal eq. (1)."""
    m, fb, props = ol.learned_match(small_img, synth.mlp_init(2), 4, 4, rms=1e9)
    assert not fb.any()
    ranges = oracle.full_ranges(48, 48, 8)
    gy, gx = oracle.domain_grid(48, 48, 8, 4)
    for q in (0, 7, 20, 35):
        y, x = ranges[q]
        r = small_img[y:y + 8, x:x + 8]
        best = None
        for j in sorted(set(props[q].tolist())):
            dd = oracle.decimate(small_img, (j // gx) * 4, (j % gx) * 4, 8)
            for t in range(8):
                for si, k in enumerate(oracle.PLAIN_K):
                    key = (oracle.eval_candidate(r, dd, t, k), j, t, si)
                    best = key if best is None or key < best else best
        assert (m["e_lit"][q], m["dom"][q], m["iso"][q], m["s_idx"][q]) == best


def test_recall():
    assert ol.recall([[1, 2], [3, 4]], [2, 5]) == 0.5
