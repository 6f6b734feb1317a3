"""GPU parity of the learned-preconditioner kernels against the FP64 oracle.

The oracle emulates the GPU's bfloat16 rounding points (the operands of the two matrix-core
layers, forward and backward-data); what remains is FP32 accumulation order, so forward
outputs, losses and gradients are compared at 1e-4 relative.  Features, diagonals and probe
statistics involve no bfloat16 and are compared at 1e-5.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import ker_to_centred, rel, small_geometry  # noqa: E402
from oracle import firm as ofirm  # noqa: E402
from oracle import pcnet as opc  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def firm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1307_5824_amd import firm as f
    return f


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _params(seed):
    p = opc.init_params(32, seed=seed, zero_last=False)
    rng = np.random.default_rng(seed + 100)
    return [(w, 0.05 * rng.standard_normal(b.shape)) for w, b in p]


def test_forward_matches_oracle(firm):
    """Network output for two random feature volumes (bf16 rounding points emulated)."""
    params = _params(1)
    f = 0.5 * np.random.default_rng(2).standard_normal((2, 32, 32, 32))
    vec = opc.flatten_params(params).astype(np.float32)
    params32 = opc.unflatten_params(vec)                 # the FP32 masters the GPU holds
    net = firm.PCNet(max_batch=2)
    net.set_params(vec)
    out = host(net.forward(dev(f)))
    for b in range(2):
        ref, _ = opc.net_forward(f[b].astype(np.float32).astype(np.float64), params32, emulate_bf16=True)
        assert rel(out[b], ref) < 1e-4


def test_loss_and_gradients_match_oracle(firm):
    """Probe loss and every parameter gradient for a batch of two samples at N = 16."""
    N = 16
    rng = np.random.default_rng(3)
    params = _params(4)
    vec = opc.flatten_params(params).astype(np.float32)
    params32 = opc.unflatten_params(vec)
    f = (0.3 * rng.standard_normal((2, 32, 32, 32))).astype(np.float32)
    A = rng.uniform(0.5, 2.0, (2, N, N, N)).astype(np.float32)
    Bs = rng.uniform(0.1, 0.6, (2, N, N, N)).astype(np.float32)
    t = rng.uniform(0.5, 3.0, (2, N, N, N)).astype(np.float32)
    sumc = np.array([1.7e3, 2.2e3])
    ker0 = np.array([2.0, 3.5])
    net = firm.PCNet(max_batch=2)
    net.set_params(vec)
    loss, g = net.loss_grad(dev(f), N, dev(t), dev(A), dev(Bs), sumc, ker0)
    ref_loss, ref_g = 0.0, None
    for b in range(2):
        # C enters the loss only through sum C: a constant field with that sum
        C = np.full((N, N, N), sumc[b] / N ** 3)
        L, grads, _ = opc.loss_and_grads(f[b].astype(np.float64), params32, N, ker0[b], t[b].astype(np.float64),
                                         A[b].astype(np.float64), Bs[b].astype(np.float64), C, emulate_bf16=True)
        ref_loss += L / 2
        flat = opc.flatten_params(grads) / 2
        ref_g = flat if ref_g is None else ref_g + flat
    assert abs(loss - ref_loss) < 1e-5 * abs(ref_loss)
    # per-layer comparison (gradients differ in scale between layers)
    k = 0
    for (w, b) in params32:
        for arr in (w, b):
            n = arr.size
            assert rel(g[k:k + n], ref_g[k:k + n]) < 1e-3, k
            k += n


@pytest.mark.parametrize("N", [16, 32])
def test_kernel_features_match_oracle(firm, N):
    R, _, _, _ = small_geometry(N, 5, 200 + N)
    Ker = ofirm.kernel_direct(N, R).real
    K32 = ker_to_centred(Ker, N).astype(np.float32)
    plan = firm.Plan(N, R)
    plan.kernel_set(dev(K32))
    feat = host(plan.kernel_features(1e-2))
    c = ofirm.circulant_first_column(K32[1:, 1:, 1:].astype(np.float64), N)
    khat = np.fft.fftn(c).real               # the Fourier multiplier of the embedded product
    ref = opc.pool_features(khat, float(K32[N, N, N]), 1e-2)
    # compared in the linear domain relative to the largest pooled value: the FP32 spectrum is
    # accurate to ~1e-6 of its maximum, which the log magnifies at small pooled values
    assert np.max(np.abs(np.exp(feat) - np.exp(ref))) < 1e-5 * np.max(np.exp(ref))


def test_forward_at_res64_matches_oracle(firm):
    """The network is fully convolutional: the same weights on a 64^3 feature grid."""
    params = _params(6)
    f = 0.5 * np.random.default_rng(7).standard_normal((1, 64, 64, 64))
    vec = opc.flatten_params(params).astype(np.float32)
    params32 = opc.unflatten_params(vec)
    net = firm.PCNet(max_batch=1)
    net.set_params(vec)
    out = host(net.forward(dev(f)))
    ref, _ = opc.net_forward(f[0].astype(np.float32).astype(np.float64), params32, emulate_bf16=True)
    assert out.shape == (1, 64, 64, 64)
    assert rel(out[0], ref) < 1e-4


def test_kernel_features_and_diagonal_at_res64(firm):
    """Features pooled to 64^3 (2 x 2 x 2 spectrum samples each at N = 64) and the diagonal
    interpolated from a 64^3 output onto N = 128."""
    N = 64
    R, _, _, _ = small_geometry(N, 4, 404)
    K32 = ker_to_centred(ofirm.kernel_direct(N, R).real, N).astype(np.float32)
    plan = firm.Plan(N, R)
    plan.kernel_set(dev(K32))
    feat = host(plan.kernel_features(1e-2, res=64))
    khat = np.fft.fftn(ofirm.circulant_first_column(K32[1:, 1:, 1:].astype(np.float64), N)).real
    ref = opc.pool_features(khat, float(K32[N, N, N]), 1e-2, g=64)
    assert np.max(np.abs(np.exp(feat) - np.exp(ref))) < 1e-5 * np.max(np.exp(ref))
    N2 = 128
    R2, _, _, _ = small_geometry(N2, 2, 405)
    plan2 = firm.Plan(N2, R2)
    K2 = np.zeros((2 * N2,) * 3, dtype=np.float32)
    K2[N2, N2, N2] = 3.0                                   # a delta kernel: Ker(0) = 3
    plan2.kernel_set(dev(K2))
    rng = np.random.default_rng(8)
    o = rng.standard_normal((64, 64, 64))
    t = rng.uniform(0.5, 6.0, (N2, N2, N2)).astype(np.float32)
    d = host(plan2.precond_from_output(dev(o), dev(t)))
    refd = opc.diagonal(o.astype(np.float32).astype(np.float64), N2, 3.0, t.astype(np.float64))
    assert rel(d, refd) < 1e-5


def test_precond_from_output_matches_oracle(firm):
    N = 32
    R, _, _, _ = small_geometry(N, 3, 7)
    plan = firm.Plan(N, R)
    plan.kernel_set(dev(ker_to_centred(ofirm.kernel_direct(N, R).real, N)))
    o = np.random.default_rng(5).standard_normal((32, 32, 32))
    t = host(plan.chan_spectrum(0.01 * plan.kernel_get()[N, N, N].item()))
    d = host(plan.precond_from_output(dev(o), dev(t)))
    ker0 = float(np.float32(ofirm.kernel_direct(N, R).real[N - 1, N - 1, N - 1]))
    ref = opc.diagonal(o.astype(np.float32).astype(np.float64), N, ker0, t)
    assert rel(d, ref) < 1e-5


def test_probe_statistics_match_oracle(firm):
    N = 16
    R, _, _, _ = small_geometry(N, 6, 9)
    Ker = ofirm.kernel_direct(N, R).real
    K32 = ker_to_centred(Ker, N).astype(np.float32)
    plan = firm.Plan(N, R)
    plan.kernel_set(dev(K32))
    probes = np.random.default_rng(11).standard_normal((3, N, N, N)).astype(np.float32)
    lam = 0.5
    A, B, sumc = plan.probe_stats(dev(probes), lam)
    Kf = K32[1:, 1:, 1:].astype(np.float64)

    def apply(v):
        return ofirm.toeplitz_apply_fft(Kf, v).real + lam * v
    Ar, Br, Cr = opc.probe_statistics(apply, N, probes.astype(np.float64))
    assert rel(host(A), Ar) < 1e-5
    assert rel(host(B), Br) < 1e-5
    assert abs(sumc - Cr.sum()) < 1e-6 * Cr.sum()


@pytest.mark.parametrize("N", [16, 32])
def test_chan_spectrum_matches_oracle(firm, N):
    """Fourier diagonal of A*A + lambda (T. Chan's circulant spectrum) vs the oracle's closed form."""
    R, _, _, _ = small_geometry(N, 7, 300 + N)
    Ker = ofirm.kernel_direct(N, R).real
    K32 = ker_to_centred(Ker, N).astype(np.float32)
    plan = firm.Plan(N, R)
    plan.kernel_set(dev(K32))
    lam = 0.37
    t = host(plan.chan_spectrum(lam))
    ref = ofirm.chan_circulant_spectrum(K32[1:, 1:, 1:].astype(np.float64), N, lam)
    assert rel(t, ref) < 1e-5


def test_kaporin_loss_and_gradients_match_oracle(firm):
    """Kaporin objective: loss and every parameter gradient for a batch of two samples at N = 16."""
    N = 16
    rng = np.random.default_rng(31)
    vec = opc.flatten_params(_params(32)).astype(np.float32)
    params32 = opc.unflatten_params(vec)
    f = (0.3 * rng.standard_normal((2, 32, 32, 32))).astype(np.float32)
    t = rng.uniform(0.5, 4.0, (2, N, N, N)).astype(np.float32)
    ker0 = np.array([2.0, 3.5])
    net = firm.PCNet(max_batch=2)
    net.set_params(vec)
    loss, g = net.loss_grad(dev(f), N, dev(t), ker0=ker0, objective="kaporin")
    ref_loss, ref_g = 0.0, None
    for b in range(2):
        L, grads, _ = opc.loss_and_grads(f[b].astype(np.float64), params32, N, ker0[b], t[b].astype(np.float64),
                                         emulate_bf16=True, objective="kaporin")
        ref_loss += L / 2
        flat = opc.flatten_params(grads) / 2
        ref_g = flat if ref_g is None else ref_g + flat
    assert abs(loss - ref_loss) < 1e-4 * abs(ref_loss) + 1e-7
    # the GPU rounds FP32 activations to BF16, the oracle FP64 ones: entries within an FP32
    # rounding of a BF16 rounding boundary round apart (2^-8 each), ~1e-3 in the gradients
    k = 0
    for w, b in params32:
        for arr in (w, b):
            n = arr.size
            assert rel(g[k:k + n], ref_g[k:k + n]) < 3e-3, k
            k += n


def _unrolled_system(N, M, seed, lam_rel=1e-2):
    from paper_1307_5824_amd import synth
    rng = np.random.default_rng(seed)
    R = synth.mixed_rotations(M, 8.0, 0.1, rng)
    Ker = ofirm.kernel_direct(N, R).real
    K32 = ker_to_centred(Ker, N).astype(np.float32)
    Kf = K32[1:, 1:, 1:].astype(np.float64)
    k0 = float(K32[N, N, N])
    lam = lam_rel * k0
    return R, K32, Kf, k0, lam, rng


@pytest.mark.parametrize("N,k,nprobes", [(16, 8, 2), (32, 6, 1), (16, 1, 1)])
def test_pcg_unrolled_matches_oracle(firm, N, k, nprobes):
    """Unrolled PCG loss and its log-d gradient (frozen-scalar reverse pass) against the FP64
    oracle on the same kernel, diagonal and probes."""
    R, K32, Kf, k0, lam, rng = _unrolled_system(N, 40, 500 + N + k)
    plan = firm.Plan(N, R)
    plan.kernel_set(dev(K32))
    t = ofirm.chan_circulant_spectrum(Kf, N, lam)
    d = (1.0 / (t + 0.2 * k0)).astype(np.float32)
    probes = rng.standard_normal((nprobes, N, N, N)).astype(np.float32)
    loss, g = plan.pcg_unrolled(dev(d), dev(probes), k, lam)
    g = host(g)

    def apply(v):
        return ofirm.toeplitz_apply_fft(Kf, v).real + lam * v
    ref_l, ref_g = 0.0, np.zeros((N, N, N))
    for z in probes.astype(np.float64):
        L, G = opc.unrolled_pcg_grad_logd(apply, d.astype(np.float64), z, k)
        ref_l += L / nprobes
        ref_g += G / nprobes
    print(f"unrolled N={N} k={k}: loss {loss:.6e} vs {ref_l:.6e}, grad rel {rel(g, ref_g):.2e}", flush=True)
    assert abs(loss - ref_l) <= 1e-4 * ref_l
    assert rel(g, ref_g) < 2e-3
    # loss only
    loss2, none = plan.pcg_unrolled(dev(d), dev(probes), k, lam, with_grad=False)
    assert none is None and abs(loss2 - loss) <= 1e-6 * loss


def test_logd_objective_gradients_match_oracle(firm):
    """Objective 2: a given log-d gradient carried through the floor, upsampling and network."""
    N = 16
    rng = np.random.default_rng(41)
    vec = opc.flatten_params(_params(42)).astype(np.float32)
    params32 = opc.unflatten_params(vec)
    f = (0.3 * rng.standard_normal((2, 32, 32, 32))).astype(np.float32)
    t = rng.uniform(0.5, 4.0, (2, N, N, N)).astype(np.float32)
    # a log-d gradient of mostly one sign, as the objectives give (a zero-mean random field would make
    # every parameter gradient a sum with heavy cancellation, which magnifies the BF16 rounding of
    # the matrix-core operands beyond the tolerance derived for it)
    G = rng.uniform(-0.5, 1.5, (2, N, N, N)).astype(np.float32)
    ker0 = np.array([2.0, 3.5])
    net = firm.PCNet(max_batch=2)
    net.set_params(vec)
    loss, g = net.loss_grad(dev(f), N, dev(t), dev(G), ker0=ker0, objective="logd")
    assert loss == 0.0
    ref_g = None
    for b in range(2):
        _, grads, _ = opc.loss_and_grads(f[b].astype(np.float64), params32, N, ker0[b], t[b].astype(np.float64),
                                         G[b].astype(np.float64), emulate_bf16=True, objective="logd")
        flat = opc.flatten_params(grads) / 2
        ref_g = flat if ref_g is None else ref_g + flat
    k, errs = 0, []
    for w, b in params32:
        for arr in (w, b):
            errs.append(rel(g[k:k + arr.size], ref_g[k:k + arr.size]))
            k += arr.size
    print("per-block gradient errors", ["%.1e" % e for e in errs], flush=True)
    assert max(errs) < 3e-3


def test_training_on_unrolled_objective_and_pcg_beats_cg(firm):
    """A short training run on the unrolled PCG objective (kernels of random view sets at N = 32)
    lowers the loss, and on a held-out view set PCG with the trained diagonal needs fewer
    iterations than plain CG to 1e-5 (FP64 refinement, precision 1)."""
    from paper_1307_5824_amd import synth, train_precond
    N, M = 32, 600
    lam_rel = 1e-2
    rng = np.random.default_rng(21)
    net = firm.PCNet(max_batch=4)
    net.set_params(train_precond.init_params(seed=5))
    data = []
    for s in range(5):
        R = synth.mixed_rotations(M, float(rng.uniform(0, 20)), 0.1, rng)
        plan = firm.Plan(N, R, lambda_relative=1, precision=1)
        plan.kernel_precompute()
        feat = plan.kernel_features(lam_rel)
        t = plan.chan_spectrum(lam_rel)
        data.append((feat, t, plan.kernel_get()[N, N, N].item(), plan))
    train, held = data[:4], data[4]
    feats = torch.stack([d[0] for d in train])
    ts = torch.stack([d[1] for d in train])
    ker0 = [d[2] for d in train]
    probes = torch.randn((2, N, N, N), device="cuda")

    def batch_loss_and_grad():
        o = net.forward(feats)
        losses, grads = [], []
        for b, (_, t, _, plan) in enumerate(train):
            d = plan.precond_from_output(o[b], t)
            L, g = plan.pcg_unrolled(d, probes, 12, lam_rel)
            losses.append(L)
            grads.append(g)
        return float(np.mean(losses)), torch.stack(grads)
    l0, _ = batch_loss_and_grad()
    for it in range(25):
        _, G = batch_loss_and_grad()
        net.train_step(feats, N, ts, G, ker0=ker0, lr=1e-5, lr_floor=1e-2, objective="logd")
    l1, _ = batch_loss_and_grad()
    print(f"unrolled loss {l0:.4e} -> {l1:.4e}", flush=True)
    assert l1 < l0
    feat, t, k0, plan = held
    atb = torch.randn((N, N, N), device="cuda")
    _, r_cg = plan.cg_solve(atb, lam_rel, 1e-5, 3000)
    d = plan.precond_from_output(net.forward(feat[None])[0], t)
    _, r_pcg = plan.cg_solve(atb, lam_rel, 1e-5, 3000, precond=d)
    _, r_chan = plan.cg_solve(atb, lam_rel, 1e-5, 3000, precond=1.0 / t)
    print("cg", r_cg["iters"], "learned pcg", r_pcg["iters"], "chan pcg", r_chan["iters"], flush=True)
    assert r_pcg["iters"] < r_cg["iters"]
