"""Pins of the learned-warm-start oracle (CPU): BF16 rounding against the two
neighbouring BF16 values, nearest neighbours against a k-d tree and a
hand-ordered line, the network through permutation weights, the loss
gradient against central differences, Adam's first step in closed form."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import learn as L


def _bf16_brute(x32: np.float32) -> int:
    """Nearest BF16 pattern by comparing the two candidates around x."""
    u = int(np.array([x32], dtype=np.float32).view(np.uint32)[0])
    lo = u >> 16
    hi = lo + 1
    v = float(x32)
    vlo = float(np.array([lo << 16], dtype=np.uint32).view(np.float32)[0])
    vhi = float(np.array([(hi << 16) & 0xFFFFFFFF], dtype=np.uint32).view(np.float32)[0])
    dlo, dhi = abs(v - vlo), abs(vhi - v)
    if dlo < dhi:
        return lo
    if dhi < dlo:
        return hi & 0xFFFF
    return lo if lo % 2 == 0 else hi & 0xFFFF


def test_bf16_rounding_is_nearest_even():
    rng = np.random.default_rng(0)
    x = (rng.normal(size=2000) * 10.0 ** rng.integers(-6, 6, size=2000)).astype(np.float32)
    # exact halfway cases, both parities, and values that carry into the exponent
    ties = np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x3FFF8000, 0x477F8000, 0x00018000],
                    dtype=np.uint32).view(np.float32)
    x = np.concatenate([x, ties, np.float32([0.0, -0.0, 1.0, 3.0e38])])
    got = L.bf16_bits(x)
    want = np.array([_bf16_brute(v) for v in x], dtype=np.uint16)
    np.testing.assert_array_equal(got, want)
    # an FP64 value is rounded to FP32 first
    assert L.bf16_bits(np.float64(1.0 + 2.0 ** -8 + 2.0 ** -40)) == L.bf16_bits(np.float32(1.0 + 2.0 ** -8))


def test_neighbours_match_a_kd_tree():
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 20, size=(300, 3))
    q, s, e = rng.uniform(-0.5, 0.5, 300), rng.uniform(3, 4, 300), rng.uniform(0.05, 0.2, 300)
    _, nb = L.features(x, q, s, e, [0, 300], rows=np.arange(0, 300, 7))
    tree = cKDTree(x)
    _, idx = tree.query(x[::7], k=17)
    for r in range(len(nb)):
        assert list(nb[r]) == [j for j in idx[r] if j != 7 * r][:16]


def test_centroid_offset_is_translation_invariant_and_sums_in_order():
    rng = np.random.default_rng(6)
    x = rng.normal(scale=5.0, size=(40, 3))
    z = np.zeros(40)
    f0, _ = L.features(x, z, z + 3.5, z, [0, 40], rows=[3, 17])
    f1, _ = L.features(x + np.array([64.0, -128.0, 32.0]), z, z + 3.5, z, [0, 40], rows=[3, 17])
    np.testing.assert_array_equal(f0, f1)
    # the offset columns agree with a centroid taken by exact rational sums
    from fractions import Fraction
    c = [float(sum(Fraction(v) for v in x[:, a]) / 40) for a in range(3)]
    got = L.bf16_value(f0[0, 115:118])
    np.testing.assert_allclose(got, (x[3] - c) / 16, rtol=2.0 ** -7)


def test_ties_go_to_the_lower_index_and_systems_are_separate():
    # atoms on a line at unit spacing: atom 5's neighbours alternate left/right
    x = np.zeros((40, 3))
    x[:, 0] = np.arange(40)
    z = np.zeros(40)
    _, nb = L.features(x, z, z + 3.5, z, [0, 20, 40], rows=[5, 25, 39])
    assert list(nb[0]) == [4, 6, 3, 7, 2, 8, 1, 9, 0, 10, 11, 12, 13, 14, 15, 16]
    assert list(nb[1]) == [24, 26, 23, 27, 22, 28, 21, 29, 20, 30, 31, 32, 33, 34, 35, 36]
    assert list(nb[2]) == list(range(38, 22, -1))


def test_feature_row_of_a_two_atom_system():
    x = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 2.0], [5.0, 5.0, 5.0]])
    q, s, e = np.array([0.25, -0.25, 0.1]), np.array([3.0, 4.0, 3.5]), np.array([0.1, 0.2, 0.05])
    fb, nb = L.features(x, q, s, e, [0, 2, 3])
    want = np.zeros(128)
    want[:10] = [0.25, -0.5, 1.0, 0.25, 0.5, 0.5, 0.75, -0.25, 0.5, 2.0]
    # centroid (0.5, 1, 1): offset (-0.5, -1, -1)/16, distance 1.5/16, n = 2
    want[115:120] = [-0.5 / 16, -1 / 16, -1 / 16, 1.5 / 16, 2 / 4096]
    np.testing.assert_array_equal(L.bf16_value(fb[0]), want)
    assert list(nb[0]) == [1] + [-1] * 15
    # a lone atom: its own parameters, no offset, n = 1
    want3 = np.zeros(128)
    want3[:3] = L.bf16([0.1, 0.0, 0.5])
    want3[119] = 1 / 4096
    np.testing.assert_array_equal(L.bf16_value(fb[2]), want3)
    assert list(nb[2]) == [-1] * 16


def _perm_params(rng):
    p1, p2 = rng.permutation(128), rng.permutation(128)
    W1 = np.zeros((128, 128))
    W1[np.arange(128), p1] = 1.0
    W2 = np.zeros((128, 128))
    W2[np.arange(128), p2] = 1.0
    W3 = L.bf16(rng.normal(size=(128, 16)))
    b3 = L.bf16(rng.normal(size=16))
    return L.pack({"W1": W1, "b1": np.zeros(128), "W2": W2, "b2": np.zeros(128), "W3": W3, "b3": b3}), p1, p2


@pytest.mark.parametrize("emulate", [True, False])
def test_forward_through_permutation_weights(emulate):
    """X = a e_k, W1 and W2 permutation matrices: H2 = a e_{p2[p1[k]]}, so
    Y = a W3[p2[p1[k]]] + b3; a transposed weight picks another row."""
    rng = np.random.default_rng(2)
    theta, p1, p2 = _perm_params(rng)
    ks = [0, 5, 77, 127]
    X = np.zeros((len(ks), 128))
    X[np.arange(len(ks)), ks] = 0.5
    Y, _ = L.forward(theta, X, emulate)
    P = L.unpack(theta)
    for r, k in enumerate(ks):
        np.testing.assert_array_equal(Y[r], 0.5 * P["W3"][p2[p1[k]]] + P["b3"])


def _random_case(seed, n=12):
    rng = np.random.default_rng(seed)
    theta = np.concatenate([rng.normal(scale=0.15, size=128 * 128), rng.normal(scale=0.1, size=128),
                            rng.normal(scale=0.1, size=128 * 128), rng.normal(scale=0.1, size=128),
                            rng.normal(scale=0.1, size=128 * 16), rng.normal(scale=0.1, size=16)])
    X = L.bf16(rng.normal(size=(n, 128)))
    T = rng.normal(size=(n, 3))
    return theta, X, T


def test_loss_gradient_matches_central_differences():
    theta, X, T = _random_case(3)
    f0, g = L.loss_grad(theta, X, T, emulate=False)
    assert f0 == pytest.approx(L.loss(theta, X, T, emulate=False), rel=1e-15)
    rng = np.random.default_rng(4)
    offsets = np.cumsum([0] + [int(np.prod(s)) for _, s in L.SHAPES])
    # W3 columns 3.. have no effect on the loss
    idx = np.concatenate([rng.integers(offsets[b], offsets[b + 1], size=12) for b in range(6)])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (L.loss(tp, X, T, emulate=False) - L.loss(tm, X, T, emulate=False)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i
    P = L.unpack(g)
    assert np.all(P["W3"][:, 3:] == 0) and np.all(P["b3"][3:] == 0)


def test_emulated_gradient_stays_close_to_the_exact_one():
    theta, X, T = _random_case(5, n=64)
    _, g = L.loss_grad(theta, X, T, emulate=False)
    _, ge = L.loss_grad(theta, X, T, emulate=True)
    cos = g @ ge / (np.linalg.norm(g) * np.linalg.norm(ge))
    assert cos > 0.999


def test_adam_first_step_and_convergence():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    th, m, v = L.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.1, eps=1e-8)
    # first step: m_hat = g and v_hat = g^2, so the move is lr * g / (|g| + eps)
    np.testing.assert_allclose(th, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=0)
    # Adam on f(t) = (t - 2)^2 reaches the minimum
    t, m, v = np.zeros(1), np.zeros(1), np.zeros(1)
    for k in range(1, 3001):
        t, m, v = L.adam(t, 2 * (t - 2.0), m, v, k, lr=0.05)
    assert abs(t[0] - 2.0) < 1e-3



@pytest.mark.parametrize("rows,seed", [(64, 1), (96, 2), (2, 3), (2050, 4)])
def test_exact_case_has_no_rounding_anywhere(rows, seed):
    """The inputs of the GPU's element-wise backward test (tests/learn_exact.py)
    must be exact: the BF16-emulated gradient equals the FP64 one bit for bit,
    the FP32 inputs hold the FP64 values, and the output layer's padding
    columns get zero gradient."""
    from tests.learn_exact import exact_case
    theta, fbits, T = exact_case(rows, seed)
    X = L.bf16_value(fbits)
    t64 = theta.astype(np.float64)
    l_e, g_e = L.loss_grad(t64, X, T.astype(np.float64), emulate=True)
    l_x, g_x = L.loss_grad(t64, X, T.astype(np.float64), emulate=False)
    np.testing.assert_array_equal(g_e, g_x)
    assert l_e == l_x
    ye, _ = L.forward(t64, X, emulate=True)
    yx, c = L.forward(t64, X, emulate=False)
    np.testing.assert_array_equal(ye, yx)
    for k in ("H1", "H2"):
        np.testing.assert_array_equal(L.bf16(c[k]), c[k])
    g = L.unpack(g_x)
    assert np.all(g["W3"][:, 3:] == 0) and np.all(g["b3"][3:] == 0)
    # the gradient is not trivially zero in any block
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert np.count_nonzero(g[k]) > 0, k
    # FP32 sums in another order give the same values: recompute with float32
    f32 = np.float32
    p = {k: v.astype(f32) for k, v in L.unpack(theta).items()}
    H1 = np.maximum(X.astype(f32) @ p["W1"] + p["b1"], 0)
    H2 = np.maximum(H1 @ p["W2"] + p["b2"], 0)
    Y = H2 @ p["W3"] + p["b3"]
    np.testing.assert_array_equal(Y.astype(np.float64), yx)
