"""Pins of the preconditioner-network oracle: convolution by its definition written as loops,
identity filters, adjoints, Parseval, and central finite differences for every gradient."""
import math

import numpy as np
import pytest

from oracle import firm as ofirm
from oracle import pcnet


def _rng(s):
    return np.random.default_rng(s)


def test_conv3d_matches_loop_definition():
    """Cross-correlation with periodic padding, written as explicit loops on a 4^3 grid."""
    rng = _rng(1)
    D, ci, co = 4, 2, 3
    x = rng.standard_normal((ci, D, D, D))
    w = rng.standard_normal((co, ci, 3, 3, 3))
    b = rng.standard_normal(co)
    y = pcnet.conv3d(x, w, b)
    for o in range(co):
        for i in range(D):
            for j in range(D):
                for k in range(D):
                    s = b[o]
                    for c in range(ci):
                        for a in range(3):
                            for bb in range(3):
                                for cc in range(3):
                                    s += w[o, c, a, bb, cc] * x[c, (i + a - 1) % D, (j + bb - 1) % D, (k + cc - 1) % D]
                    assert abs(s - y[o, i, j, k]) < 1e-12


def test_conv3d_identity_filter():
    rng = _rng(2)
    x = rng.standard_normal((3, 5, 5, 5))
    w = np.zeros((3, 3, 3, 3, 3))
    for c in range(3):
        w[c, c, 1, 1, 1] = 1.0
    assert np.allclose(pcnet.conv3d(x, w, np.zeros(3)), x)


def test_conv3d_backward_finite_differences():
    rng = _rng(3)
    D, ci, co = 4, 2, 3
    x = rng.standard_normal((ci, D, D, D))
    w = rng.standard_normal((co, ci, 3, 3, 3))
    b = rng.standard_normal(co)
    dy = rng.standard_normal((co, D, D, D))
    dx, dw, db = pcnet.conv3d_backward(x, w, dy)
    f = lambda x_, w_, b_: float(np.sum(dy * pcnet.conv3d(x_, w_, b_)))  # noqa: E731
    h = 1e-6
    for idx in [(0, 1, 2, 3), (1, 0, 0, 0)]:
        e = np.zeros_like(x); e[idx] = h
        assert abs((f(x + e, w, b) - f(x - e, w, b)) / (2 * h) - dx[idx]) < 1e-6 * (1 + abs(dx[idx]))
    for idx in [(2, 1, 0, 2, 1), (0, 0, 1, 1, 1)]:
        e = np.zeros_like(w); e[idx] = h
        assert abs((f(x, w + e, b) - f(x, w - e, b)) / (2 * h) - dw[idx]) < 1e-6 * (1 + abs(dw[idx]))
    e = np.zeros_like(b); e[1] = h
    assert abs((f(x, w, b + e) - f(x, w, b - e)) / (2 * h) - db[1]) < 1e-6 * (1 + abs(db[1]))


@pytest.mark.parametrize("G", [32, 64])
def test_upsample_properties(G):
    rng = _rng(4)
    s = rng.standard_normal((G, G, G))
    assert np.allclose(pcnet.upsample(s, G), s)                         # N = G samples the grid
    assert np.allclose(pcnet.upsample(np.full((G, G, G), 2.5), 64), 2.5)
    up2 = pcnet.upsample(s, 2 * G)                                       # N = 2G: even points hit the
    assert np.allclose(up2[::2, ::2, ::2], s)                            # grid, odd ones are midpoints
    assert np.allclose(up2[1::2, ::2, ::2], 0.5 * (s + np.roll(s, -1, axis=0)))
    g = rng.standard_normal((16, 16, 16))
    lhs = np.sum(pcnet.upsample(s, 16) * g)
    rhs = np.sum(s * pcnet.upsample_adjoint(g, 16, G))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    ss = pcnet.symmetrise(s)
    assert np.allclose(ss, np.roll(ss[::-1, ::-1, ::-1], 1, axis=(0, 1, 2)))
    assert np.allclose(pcnet.symmetrise(ss), ss)
    up = pcnet.upsample(ss, 16)                                           # symmetric stays symmetric
    assert np.allclose(up, np.roll(up[::-1, ::-1, ::-1], 1, axis=(0, 1, 2)))


def test_probe_loss_is_parseval_of_the_residual():
    """sum (d^2 A - 2 d B + C) / sum C equals sum ||P u - z||^2 / sum ||z||^2 computed in real space."""
    rng = _rng(5)
    N = 8
    R = np.stack([np.eye(3)])
    Ker = ofirm.kernel_direct(N, R).real
    lam = 3.0

    def apply(v):
        return ofirm.toeplitz_apply_fft(Ker, v).real + lam * v
    probes = rng.standard_normal((3, N, N, N))
    A, B, C = pcnet.probe_statistics(apply, N, probes)
    d = rng.uniform(0.01, 0.1, (N, N, N))
    d = 0.5 * (d + np.roll(d[::-1, ::-1, ::-1], 1, axis=(0, 1, 2)))
    num = sum(np.sum((pcnet.precond_apply(d, apply(z)) - z) ** 2) for z in probes)
    den = sum(np.sum(z ** 2) for z in probes)
    assert abs(pcnet.probe_loss(d, A, B, C) - num / den) < 1e-10 * (num / den)


def test_full_chain_gradients_finite_differences():
    """Loss through network, symmetrisation, upsampling, exp and the probe quadratic: central
    differences on a few parameters of every layer."""
    rng = _rng(6)
    N, C = 8, 2
    G = pcnet.G
    params = pcnet.init_params(C, seed=1, zero_last=False)
    params = [(w * 0.3, b + 0.01 * rng.standard_normal(b.shape)) for w, b in params]
    f = 0.2 * rng.standard_normal((G, G, G))
    A = rng.uniform(0.5, 2.0, (N, N, N))
    B = rng.uniform(0.1, 0.5, (N, N, N))
    Cs = rng.uniform(0.5, 1.0, (N, N, N))
    t = rng.uniform(0.5, 2.0, (N, N, N))
    t = 0.5 * (t + np.roll(t[::-1, ::-1, ::-1], 1, axis=(0, 1, 2)))
    ker0 = 3.0
    L, grads, _ = pcnet.loss_and_grads(f, params, N, ker0, t, A, B, Cs)
    # a step of 1e-6 stays clear of the ReLU kinks (a few dozen pre-activations lie within 1e-4
    # of zero); FP64 round-off then limits the agreement to ~1e-5 relative
    h = 1e-6
    for layer, idx in [(0, (1, 0, 0, 1, 2)), (1, (0, 1, 2, 2, 0)), (2, (1, 1, 1, 1, 1)), (3, (0, 1, 0, 0, 0))]:
        w, b = params[layer]
        wp = [list(p) for p in params]
        wp[layer][0] = w.copy(); wp[layer][0][idx] += h
        lp, _, _ = pcnet.loss_and_grads(f, [tuple(p) for p in wp], N, ker0, t, A, B, Cs)
        wp[layer][0] = w.copy(); wp[layer][0][idx] -= h
        lm, _, _ = pcnet.loss_and_grads(f, [tuple(p) for p in wp], N, ker0, t, A, B, Cs)
        fd = (lp - lm) / (2 * h)
        # absolute floor: FP64 round-off of a loss of order 1 divided by the step
        assert abs(fd - grads[layer][0][idx]) <= 5e-5 * abs(fd) + 5e-10, (layer, fd, grads[layer][0][idx])
    wp = [list(p) for p in params]
    b3 = params[3][1]
    wp[3][1] = b3 + h
    lp, _, _ = pcnet.loss_and_grads(f, [tuple(p) for p in wp], N, ker0, t, A, B, Cs)
    wp[3][1] = b3 - h
    lm, _, _ = pcnet.loss_and_grads(f, [tuple(p) for p in wp], N, ker0, t, A, B, Cs)
    assert abs((lp - lm) / (2 * h) - grads[3][1][0]) <= 5e-5 * abs(grads[3][1][0]) + 1e-12


def test_untrained_network_is_a_constant_floor():
    """With the last layer's weights at zero and its bias log(mu), d = 1 / (t + mu Ker(0))."""
    rng = _rng(7)
    G = pcnet.G
    params = pcnet.init_params(4, seed=2, floor=0.25)
    f = rng.standard_normal((G, G, G))
    o, _ = pcnet.net_forward(f, params)
    assert np.allclose(o, np.log(0.25))
    t = rng.uniform(0.1, 3.0, (16, 16, 16))
    d = pcnet.diagonal(o, 16, 2.0, t)
    assert np.allclose(d, 1.0 / (t + 0.5))


def test_bf16_rounding():
    """Round-to-nearest-even to 8 significant bits: exact for representable values, ties to even."""
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 0.0])
    got = pcnet.bf16(vals)
    assert list(got) == [1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6, -2.5, 0.0]


def test_flatten_roundtrip():
    params = pcnet.init_params(32, seed=3, zero_last=False)
    vec = pcnet.flatten_params(params)
    assert vec.size == 57121
    back = pcnet.unflatten_params(vec)
    for (w, b), (w2, b2) in zip(params, back):
        assert np.array_equal(w, w2) and np.array_equal(b, b2)


def test_kaporin_loss_minimum_and_scale_invariance():
    """log(mean(d t)) - mean(log(d t)) >= 0 (AM-GM), zero iff d is proportional to 1 / t, and
    unchanged when d is scaled."""
    rng = _rng(8)
    t = rng.uniform(0.1, 10.0, (6, 6, 6))
    d = rng.uniform(0.1, 10.0, (6, 6, 6))
    assert pcnet.kaporin_loss(d, t) > 0
    assert abs(pcnet.kaporin_loss(3.7 / t, t)) < 1e-14
    assert abs(pcnet.kaporin_loss(5.0 * d, t) - pcnet.kaporin_loss(d, t)) < 1e-13
    # gradient with respect to log d: central differences
    g = pcnet.kaporin_grad_logd(d, t)
    h = 1e-6
    for idx in [(0, 0, 0), (2, 3, 1), (5, 5, 4)]:
        e = np.zeros_like(d); e[idx] = h
        fd = (pcnet.kaporin_loss(d * np.exp(e), t) - pcnet.kaporin_loss(d * np.exp(-e), t)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * (abs(g[idx]) + 1e-9)
    assert abs(g.sum()) < 1e-12       # scale invariance: the gradient sums to zero


def test_full_chain_gradients_kaporin():
    """Network, symmetrisation, upsampling and exp under the Kaporin objective: central
    differences on a parameter of every layer."""
    rng = _rng(9)
    N, C = 8, 2
    params = pcnet.init_params(C, seed=3, zero_last=False)
    params = [(w * 0.3, b + 0.01 * rng.standard_normal(b.shape)) for w, b in params]
    f = 0.2 * rng.standard_normal((pcnet.G,) * 3)
    t = rng.uniform(0.5, 2.0, (N, N, N))
    t = 0.5 * (t + np.roll(t[::-1, ::-1, ::-1], 1, axis=(0, 1, 2)))
    args = (N, 2.0, t)
    L, grads, _ = pcnet.loss_and_grads(f, params, *args, objective="kaporin")
    h = 1e-6
    for layer, idx in [(0, (1, 0, 0, 1, 2)), (1, (0, 1, 2, 2, 0)), (2, (1, 1, 1, 1, 1)), (3, (0, 1, 0, 0, 0))]:
        w = params[layer][0]
        wp = [list(p) for p in params]
        wp[layer][0] = w.copy(); wp[layer][0][idx] += h
        lp, _, _ = pcnet.loss_and_grads(f, [tuple(p) for p in wp], *args, objective="kaporin")
        wp[layer][0] = w.copy(); wp[layer][0][idx] -= h
        lm, _, _ = pcnet.loss_and_grads(f, [tuple(p) for p in wp], *args, objective="kaporin")
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grads[layer][0][idx]) <= 5e-5 * abs(fd) + 1e-12, (layer, fd, grads[layer][0][idx])


@pytest.mark.parametrize("N2,g", [(32, 8), (32, 16), (64, 32)])
def test_pool_features_block_loop(N2, g):
    """Pooled features against an explicit loop over the coarse cells: coarse centred index u
    averages |K^| over the fine frequencies q_d in [(u_d - g/2) s, (u_d - g/2) s + s), s = 2N/g,
    read from the FFT-order spectrum at q mod 2N."""
    rng = np.random.default_rng(71)
    khat = rng.standard_normal((N2, N2, N2))
    ker0, lam = 3.7, 0.02
    s = N2 // g
    ref = np.empty((g, g, g))
    idx = [np.arange((u - g // 2) * s, (u - g // 2) * s + s) % N2 for u in range(g)]
    for u1 in range(g):
        for u2 in range(g):
            for u3 in range(g):
                blk = np.abs(khat[np.ix_(idx[u1], idx[u2], idx[u3])])
                ref[u1, u2, u3] = math.log(blk.sum() / s ** 3 / ker0 + lam)
    got = pcnet.pool_features(khat, ker0, lam, g)
    assert np.max(np.abs(got - ref)) <= 1e-12


# ------------------------------------------------ unrolled PCG objective --

def _toeplitz_system(N, M, seed, lam_rel=0.01):
    rng = _rng(seed)
    from paper_1307_5824_amd import synth
    R = synth.haar_rotations(M, rng)
    Ker = ofirm.kernel_direct(N, R).real
    lam = lam_rel * Ker[N - 1, N - 1, N - 1]

    def apply(v):
        return ofirm.toeplitz_apply_fft(Ker, v).real + lam * v
    return Ker, lam, apply, rng


def test_unrolled_loss_is_the_krylov_energy_error():
    """The k-step PCG iterate is the energy-norm minimiser over the preconditioned Krylov space
    span{(P T)^j P b}: the loss equals the error of that minimiser, computed by a dense
    least-squares solve in the T inner product (a definition independent of the recursion)."""
    N, k = 8, 5
    Ker, lam, apply, rng = _toeplitz_system(N, 6, 11)
    t = ofirm.chan_circulant_spectrum(Ker, N, lam)
    d = 1.0 / (t + 0.1 * Ker[N - 1, N - 1, N - 1])
    z = rng.standard_normal((N, N, N))
    b = apply(z)
    V = [pcnet.precond_apply(d, b)]
    for _ in range(k - 1):
        V.append(pcnet.precond_apply(d, apply(V[-1])))
    V = np.stack([v.reshape(-1) / np.linalg.norm(v) for v in V], axis=1)
    TV = np.stack([apply(V[:, j].reshape(z.shape)).reshape(-1) for j in range(k)], axis=1)
    c = np.linalg.solve(V.T @ TV, V.T @ b.reshape(-1))
    e = z.reshape(-1) - V @ c
    ref = float(e @ apply(e.reshape(z.shape)).reshape(-1) / np.sum(z * b))
    got = pcnet.unrolled_pcg_loss(apply, d, z, k)
    assert abs(got - ref) <= 1e-8 * ref


def test_unrolled_gradient_finite_differences():
    """The frozen-scalar reverse pass equals central differences of the loss along random even
    directions in log d (the loss of the recursion itself, so this pins the envelope argument)."""
    N, k = 8, 6
    Ker, lam, apply, rng = _toeplitz_system(N, 5, 12)
    t = ofirm.chan_circulant_spectrum(Ker, N, lam)
    d = 1.0 / (t + 0.2 * Ker[N - 1, N - 1, N - 1])
    z = rng.standard_normal((N, N, N))
    L, g = pcnet.unrolled_pcg_grad_logd(apply, d, z, k)
    assert abs(L - pcnet.unrolled_pcg_loss(apply, d, z, k)) <= 1e-12 * L
    # P is invariant to scaling d, so the gradient in log d sums to zero
    assert abs(g.sum()) <= 1e-6 * np.abs(g).sum()
    h = 1e-5
    for _ in range(3):
        v = rng.standard_normal(d.shape)
        v = 0.5 * (v + np.roll(v[::-1, ::-1, ::-1], 1, axis=(0, 1, 2)))
        fd = (pcnet.unrolled_pcg_loss(apply, d * np.exp(h * v), z, k)
              - pcnet.unrolled_pcg_loss(apply, d * np.exp(-h * v), z, k)) / (2 * h)
        assert abs(fd - np.sum(g * v)) <= 2e-3 * abs(fd), (fd, np.sum(g * v))


def test_unrolled_loss_one_step_with_exact_inverse():
    """On a circulant operator with d its inverse spectrum, one PCG step is exact: loss 0 and zero
    gradient."""
    N = 8
    rng = _rng(13)
    s = rng.uniform(0.5, 3.0, (N, N, N))
    s = 0.5 * (s + np.roll(s[::-1, ::-1, ::-1], 1, axis=(0, 1, 2)))

    def apply(v):
        return pcnet.precond_apply(s, v)
    z = rng.standard_normal((N, N, N))
    L, g = pcnet.unrolled_pcg_grad_logd(apply, 1.0 / s, z, 1)
    assert L <= 1e-24 and np.max(np.abs(g)) <= 1e-12


def test_full_chain_gradients_given_logd():
    """Network, symmetrisation, upsampling and the floor under a loss whose log-d gradient is
    given: the chain equals central differences of sum(G log d) in the parameters."""
    rng = _rng(14)
    N, C = 8, 2
    params = pcnet.init_params(C, seed=4, zero_last=False)
    params = [(w * 0.3, b + 0.01 * rng.standard_normal(b.shape)) for w, b in params]
    f = 0.2 * rng.standard_normal((pcnet.G,) * 3)
    t = rng.uniform(0.5, 2.0, (N, N, N))
    t = 0.5 * (t + np.roll(t[::-1, ::-1, ::-1], 1, axis=(0, 1, 2)))
    Gl = rng.standard_normal((N, N, N))
    ker0 = 2.0

    def lin(ps):
        o, _ = pcnet.net_forward(f, ps)
        return float(np.sum(Gl * np.log(pcnet.diagonal(o, N, ker0, t))))
    _, grads, _ = pcnet.loss_and_grads(f, params, N, ker0, t, Gl, objective="logd")
    h = 1e-6
    for layer, idx in [(0, (1, 0, 0, 1, 2)), (2, (1, 1, 1, 1, 1)), (3, (0, 1, 0, 0, 0))]:
        w = params[layer][0]
        wp = [list(p) for p in params]
        wp[layer][0] = w.copy(); wp[layer][0][idx] += h
        lp = lin([tuple(p) for p in wp])
        wp[layer][0] = w.copy(); wp[layer][0][idx] -= h
        lm = lin([tuple(p) for p in wp])
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grads[layer][0][idx]) <= 5e-5 * abs(fd) + 1e-12, (layer, fd, grads[layer][0][idx])
