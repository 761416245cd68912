"""Pins of the FP64 surrogate reference (oracle/surrogate.py): values fixed by
hand counting, closed forms and finite differences, not by re-typing the
reference's formulas."""
import numpy as np

from oracle import surrogate as S


def _uniform_levels(L, n0):
    return S.pyramid(np.full((1 << L,) * 3, n0))


def test_feature_stencils_of_a_uniform_field_at_the_corners():
    """Uniform n0 on 256^3: inside the box every feature is ln n0, outside
    ln 1e-10.  Counted by hand: at the low corner the stencil 2A-1 .. 2A+2
    with A = 0 keeps 0, 1, 2 per axis (27 cells) for l >= 2, 0 and 1 (8
    cells) at l = 1 and the root alone at l = 0; the high corner keeps the
    last three cells per axis; the centre cell (128, 128, 128) has A = 1 at
    level 1, so its level-2 stencil is 1 .. 4 of 0 .. 3 (27 cells inside),
    and all 64 cells are inside for l >= 3."""
    L, n0 = 8, 7.5
    lv = _uniform_levels(L, n0)
    n = 1 << L
    cells = np.array([0, n ** 3 - 1, (n // 2) * (n * n + n + 1)])
    f = S.features(lv, cells)
    inside = np.isclose(f, np.log(n0), rtol=0, atol=1e-12)
    outside = np.isclose(f, np.log(1e-10), rtol=0, atol=1e-12)
    assert (inside | outside).all()
    counts = inside.reshape(3, 9, 64).sum(axis=2)
    assert counts[0].tolist() == [1, 8] + [27] * 7
    assert counts[1].tolist() == [1, 8] + [27] * 7
    assert counts[2].tolist() == [1, 8, 27] + [64] * 6
    # low corner, level 5: offsets with every s >= 1 are inside
    sel = [s for s in range(64) if (s & 3) >= 1 and ((s >> 2) & 3) >= 1 and (s >> 4) >= 1]
    assert inside[0, 5 * 64 + np.array(sel)].all()


def test_feature_of_a_point_mass_is_diluted_by_eight_per_level():
    """One non-zero leaf v at (x0, y0, z0) of a 256^3 grid: the level-l cell
    holding it has density v 8^-(8-l); for the target at (x0, y0, z0) that
    cell is the child (x0 >> (8-l)) - 2 A + 1 of the stencil, and every
    other stencil cell is empty."""
    L, v = 8, 3.0e6
    x0, y0, z0 = 100, 37, 201
    field = np.zeros((1 << L,) * 3)
    field[z0, y0, x0] = v
    lv = S.pyramid(field)
    f = S.features(lv, np.array([(z0 * 256 + y0) * 256 + x0]))[0]
    for l in range(9):
        A = np.array([x0, y0, z0]) >> (L - l + 1)
        s = (np.array([x0, y0, z0]) >> (L - l)) - (2 * A - 1)
        k = l * 64 + s[0] + 4 * s[1] + 16 * s[2]
        assert abs(f[k] - np.log(v * 8.0 ** (l - L))) < 1e-9
        others = np.delete(f[l * 64:(l + 1) * 64], k - l * 64)
        assert np.allclose(others, np.log(1e-10), atol=1e-12)


def test_feature_scaling():
    lv = _uniform_levels(8, 2.0)
    f0 = S.features(lv, np.array([12345]))
    f1 = S.features(lv, np.array([12345]), in_shift=1.5, in_scale=4.0)
    assert np.allclose(f1, (f0 - 1.5) / 4.0, atol=1e-14)


def test_mlp_gradients_match_central_finite_differences():
    rng = np.random.default_rng(0)
    W, D, n = 5, 3, 7
    params = [rng.normal(0, 0.1, s) for s in S.param_shapes(W, D)]
    X = rng.normal(0, 1, (n, S.N_FEAT))
    T = rng.normal(0, 1, (n, D))
    Y, cache = S.forward(params, X)
    g = S.flatten(S.backward(params, cache, Y, T))
    p = S.flatten(params)
    h = 1e-6
    idx = np.concatenate([rng.choice(S.N_FEAT * W, 40, replace=False),  # W1
                          np.arange(S.N_FEAT * W, p.size)])             # everything else
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp = S.mse(S.forward(S.unflatten(pp, W, D), X)[0], T)
        lm = S.mse(S.forward(S.unflatten(pm, W, D), X)[0], T)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_first_step_closed_form():
    """With zero moments, bias correction makes the first step
    -lr g / (|g| + eps) whatever the gradient's size."""
    p = np.array([1.0, -2.0, 0.5, 3.0])
    g = np.array([1e-3, -7.0, 0.0, 2e5])
    p1, m, v = S.adam_step(p, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_hand_built_network():
    """W1 routes feature 3 to hidden unit 0, W2 passes unit 0 through, W3
    copies it to output 1 with bias 0.25: y1 = relu(x3) + 0.25, others 0.25."""
    W, D = 4, 2
    W1 = np.zeros((S.N_FEAT, W)); W1[3, 0] = 1.0
    W2 = np.zeros((W, W)); W2[0, 0] = 1.0
    W3 = np.zeros((W, D)); W3[0, 1] = 1.0
    params = [W1, np.zeros(W), W2, np.zeros(W), W3, np.full(D, 0.25)]
    X = np.zeros((3, S.N_FEAT)); X[:, 3] = [2.0, -1.0, 0.5]
    Y, _ = S.forward(params, X)
    assert np.allclose(Y[:, 1], [2.25, 0.25, 0.75]) and np.allclose(Y[:, 0], 0.25)


def test_bf16_rounding():
    a = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 3.0e-20, -5.5])
    r = S.bf16_round(a)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: to even (1); 1 + 3 2^-9 rounds up
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7 and r[4] == -5.5
    assert abs(r[3] / 3.0e-20 - 1) < 2 ** -8
