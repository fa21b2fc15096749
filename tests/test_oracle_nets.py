"""Pins of the oracle's networks for the biased initial-state selection and the
actor warm start (paper Sec. II, III-C/D): the packed-parameter perceptron
against closed forms and the composition of affine maps, the top-N selection
against a brute-force sort, and the actor rollout against constant controls
and an exact linear-feedback closed loop."""
import numpy as np
import pytest

from paper_2602_19699_amd import inputs as I

from lq_dense import unpack_lq

LQ, PM, P3 = I.SYS_LQ, I.SYS_POINT_MASS, I.SYS_PLANAR3


def layers(params, in_dim, width, depth, out_dim):
    """Split packed parameters into [(W, b), ...] (row-major, y = x W + b)."""
    p = np.asarray(params, dtype=np.float64)
    out, c, fan = [], 0, in_dim
    for _ in range(depth):
        W = p[c:c + fan * width].reshape(fan, width); c += fan * width
        b = p[c:c + width]; c += width
        out.append((W, b))
        fan = width
    W = p[c:c + fan * out_dim].reshape(fan, out_dim); c += fan * out_dim
    out.append((W, p[c:c + out_dim])); c += out_dim
    assert c == len(p)
    return out


def pack(ls):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in ls]).astype(np.float32)


def net(orc, in_dim, width, depth, out_dim, params, act=0, out_act=0, scale=1.0):
    return orc.Net(in_dim, width, depth, out_dim, act, out_act, scale, params)


def test_zero_weights_give_the_output_map_of_the_bias(orc):
    b = np.array([-50.0, -1.0, 0.0, 1.0, 50.0])
    for out_act, ref in [(0, b), (1, 2.5 * np.tanh(b)), (2, np.logaddexp(0.0, b))]:
        ls = [(np.zeros((3, 8)), np.zeros(8)), (np.zeros((8, 5)), b)]
        y = orc.mlp_forward(net(orc, 3, 8, 1, 5, pack(ls), out_act=out_act, scale=2.5), np.random.rand(4, 3))
        np.testing.assert_allclose(y, np.tile(ref, (4, 1)), rtol=1e-15, atol=0)


@pytest.mark.parametrize("act", [1, 2], ids=["elu", "relu"])
def test_positive_network_is_the_composed_affine_map(orc, act):
    # nonnegative weights, inputs and biases keep every pre-activation positive,
    # where ELU and ReLU are the identity: the network is one affine map
    rng = np.random.default_rng(7)
    dims = [5, 16, 16, 16, 3]
    ls = [(rng.uniform(0, 0.3, (dims[i], dims[i + 1])), rng.uniform(0.01, 0.2, dims[i + 1])) for i in range(4)]
    params = pack(ls)
    ls = layers(params, 5, 16, 3, 3)  # the float32-rounded values
    A = ls[0][0] @ ls[1][0] @ ls[2][0] @ ls[3][0]
    c = ((ls[0][1] @ ls[1][0] + ls[1][1]) @ ls[2][0] + ls[2][1]) @ ls[3][0] + ls[3][1]
    x = rng.uniform(0, 1, (50, 5))
    y = orc.mlp_forward(net(orc, 5, 16, 3, 3, params, act=act), x)
    np.testing.assert_allclose(y, x @ A + c, rtol=1e-13)


def test_single_neuron_closed_forms(orc):
    x = np.linspace(-3, 3, 13)[:, None]
    w0, b0, w1, b1 = 0.7, -0.2, -1.3, 0.4
    ls = [(np.array([[w0]]), np.array([b0])), (np.array([[w1]]), np.array([b1]))]
    z = np.float32(w0) * x[:, 0] + np.float32(b0)
    for act, f in [(0, np.tanh), (1, lambda v: np.where(v > 0, v, np.expm1(v))), (2, lambda v: np.maximum(v, 0))]:
        y = orc.mlp_forward(net(orc, 1, 1, 1, 1, pack(ls), act=act), x)[:, 0]
        np.testing.assert_allclose(y, np.float32(w1) * f(z) + np.float32(b1), rtol=1e-14, atol=1e-15)


def test_hidden_unit_permutation_invariance(orc):
    rng = np.random.default_rng(3)
    params = I.mlp_params(6, 32, 2, 2, seed=4)
    ls = layers(params, 6, 32, 2, 2)
    P1, P2 = rng.permutation(32), rng.permutation(32)
    perm = [(ls[0][0][:, P1], ls[0][1][P1]), (ls[1][0][P1][:, P2], ls[1][1][P2]), (ls[2][0][P2], ls[2][1])]
    x = rng.normal(size=(40, 6))
    a = orc.mlp_forward(net(orc, 6, 32, 2, 2, params), x)
    b = orc.mlp_forward(net(orc, 6, 32, 2, 2, pack(perm)), x)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)


def test_top_n_definition(orc):
    rng = np.random.default_rng(5)
    s = rng.integers(0, 20, 300).astype(np.float64)  # many ties
    s[[3, 77]] = np.nan
    s[[5, 9]] = [0.0, -0.0]
    for N in (0, 1, 17, 150, 298, 300):
        brute = sorted(range(300), key=lambda i: (np.isnan(s[i]), -(s[i] if not np.isnan(s[i]) else 0), i))[:N]
        np.testing.assert_array_equal(orc.top_n(s, N), np.sort(brute))
    assert set(orc.top_n(s, 300)[-2:]) <= set(range(300))
    assert 3 not in orc.top_n(s, 298) and 77 not in orc.top_n(s, 298)
    # -0 and +0 tie: the lower index wins
    z = np.array([1.0, -0.0, 0.0, -1.0])
    np.testing.assert_array_equal(orc.top_n(z, 2), [0, 1])


def test_bic_select_takes_the_most_uncertain(orc):
    x, T, T_max = I.bic_candidates("pm16k", 1000, seed=11)
    assert T_max == 100 and T.min() >= 1 and T.max() <= 100
    params = I.mlp_params(5, 32, 2, 1, seed=8)
    nt = net(orc, 5, 32, 2, 1, params, act=0, out_act=2)
    sc, sel = orc.bic_select(nt, x, T, T_max, 100)
    assert np.all(sc > 0) and len(sel) == 100 and np.all(np.diff(sel) > 0)
    rest = np.setdiff1d(np.arange(1000), sel)
    assert sc[sel].min() >= sc[rest].max()
    # the time input of candidate i is (T_max - T_i) / T_max
    ref = orc.mlp_forward(nt, np.concatenate([x, ((100 - T) / 100.0)[:, None]], axis=1))[:, 0]
    np.testing.assert_array_equal(sc, ref)


def test_constant_actor_rolls_out_constant_controls(orc):
    p = I.point_mass_params(0)
    x0 = I.point_mass_x0(5, seed=9)
    b = np.array([0.3, -0.8])
    ls = [(np.zeros((5, 32)), np.zeros(32)), (np.zeros((32, 2)), b)]
    T = np.array([100, 1, 37, 0, 101], np.int32)  # the last two are outside 1..100
    U, X = orc.actor_rollout(PM, p, net(orc, 5, 32, 1, 2, pack(ls), out_act=1, scale=4.0), x0, 100, T=T)
    for i in range(5):
        if T[i] < 1 or T[i] > 100:
            assert np.all(U[i] == 0) and np.all(X[i] == 0)
            continue
        u = 4.0 * np.tanh(np.float32(b).astype(np.float64))
        np.testing.assert_allclose(U[i, :T[i]], np.tile(u, (T[i], 1)), rtol=1e-15, atol=0)
        assert np.all(U[i, T[i]:] == 0) and np.all(X[i, T[i] + 1:] == 0)
        d, _ = orc.check_trajectory(PM, p, X[i, :T[i] + 1], U[i, :T[i]])
        assert d == 0.0 and np.array_equal(X[i, 0], x0[i])


def test_linear_feedback_actor_gives_the_closed_loop(orc):
    # relu(z) - relu(-z) = z: a one-hidden-layer ReLU network with W_0 = [I, -I]
    # and W_out = [-K'; K'] is the feedback u = -K x (tau has zero weight)
    p = I.lq_random(4, 2, seed=2)
    A, B, *_ = unpack_lq(p)
    K = np.random.default_rng(1).normal(size=(2, 4)) * 0.5
    W0 = np.zeros((5, 32))
    W0[:4, :4], W0[:4, 4:8] = np.eye(4), -np.eye(4)
    Wo = np.zeros((32, 2))
    Wo[:4], Wo[4:8] = -K.T, K.T
    ls = [(W0, np.zeros(32)), (Wo, np.zeros(2))]
    params = pack(ls)
    Kf = layers(params, 5, 32, 1, 2)[1][0][4:8].T  # K as rounded to FP32
    x0 = I.lq_x0(3, 4, seed=4)
    U, X = orc.actor_rollout(LQ, p, net(orc, 5, 32, 1, 2, params, act=2), x0, 30)
    Acl = A - B @ Kf
    for i in range(3):
        for k in range(31):
            np.testing.assert_allclose(X[i, k], np.linalg.matrix_power(Acl, k) @ x0[i], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(U[i, 5], -Kf @ X[i, 5], rtol=1e-13, atol=1e-15)


def test_actor_time_input(orc):
    # an actor that outputs its time input: u_k = tau_k = (T_max - T_b + k) / T_max
    p = I.lq_random(2, 1, seed=0)
    W0 = np.zeros((3, 32))
    W0[2, 0] = 1.0
    Wo = np.zeros((32, 1))
    Wo[0, 0] = 1.0
    params = pack([(W0, np.zeros(32)), (Wo, np.zeros(1))])
    T = np.array([10, 4], np.int32)
    U, _ = orc.actor_rollout(LQ, p, net(orc, 3, 32, 1, 1, params, act=2), I.lq_x0(2, 2), 10, T=T)
    np.testing.assert_allclose(U[0, :, 0], np.arange(10) / 10, rtol=0, atol=1e-16)
    np.testing.assert_allclose(U[1, :4, 0], (6 + np.arange(4)) / 10, rtol=0, atol=1e-16)
