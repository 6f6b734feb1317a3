"""The Fourier-space damping regularizer (section 5) on the GPU against the FP64 oracle.

The operator is A*A + lam + mu L_p, with L_p the zero-padded 2N embedding of w^p, w the symbol of
the 7-point negative Laplacian (pinned on the CPU against the stencil itself): the oracle applies
Ker + mu r_p through the circulant embedding, r_p = regularizer_kernel(N, p).  FP32 products to
1e-5, FP64 to 1e-12, Chan's spectrum to 1e-5, solves certified by the oracle's residual.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import ker_to_centred, rel, small_geometry  # noqa: E402
from oracle import firm as ofirm  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def firm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1307_5824_amd import firm as f
    return f


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def _system(N, M, seed):
    R, sh, grp, table = small_geometry(N, M, seed, groups=2)
    h = ofirm.ctf_weights(N, M, grp, table)
    Ker = ofirm.kernel_direct(N, R, h).real
    K32 = ker_to_centred(Ker, N).astype(np.float32)
    return R, K32, K32[1:, 1:, 1:].astype(np.float64)


@pytest.mark.parametrize("N,order", [(16, 1), (16, 2), (32, 1), (16, 3)])
def test_regularized_product_matches_oracle(firm, N, order):
    R, K32, Kf = _system(N, 4 if N == 16 else 3, 600 + N + order)
    ker0 = float(K32[N, N, N])
    lam, mu = 1e-2 * ker0, 3e-3 * ker0
    plan = firm.Plan(N, R)
    plan.kernel_set(dev(K32))
    plan.set_regularizer(order, mu)
    x = np.random.default_rng(order).standard_normal((N, N, N)).astype(np.float32)
    y = plan.apply_AtA(dev(x), lam).cpu().numpy()
    x64 = x.astype(np.float64)
    ref = ofirm.toeplitz_apply_fft(Kf + mu * ofirm.regularizer_kernel(N, order), x64).real + lam * x64
    print(f"N={N} order {order}: FP32 product rel err {rel(y, ref):.2e}", flush=True)
    assert rel(y, ref) < 1e-5
    y64 = plan.apply_AtA_f64(dev(x, torch.float64), lam).cpu().numpy()
    assert rel(y64, ref) < 1e-12
    # the damping term alone: the difference to the unregularized product
    plan.set_regularizer(0, 0.0)
    y0 = plan.apply_AtA(dev(x), lam).cpu().numpy().astype(np.float64)
    d_ref = mu * ofirm.regularizer_apply(x64, order)
    assert rel(y - y0, d_ref) < 1e-4


def test_regularizer_before_and_after_the_kernel(firm):
    N = 16
    R, K32, _ = _system(N, 4, 610)
    x = dev(np.random.default_rng(1).standard_normal((N, N, N)))
    p1 = firm.Plan(N, R)
    p1.set_regularizer(2, 5.0)
    p1.kernel_set(dev(K32))
    p2 = firm.Plan(N, R)
    p2.kernel_set(dev(K32))
    p2.set_regularizer(2, 5.0)
    assert torch.equal(p1.apply_AtA(x, 1.0), p2.apply_AtA(x, 1.0))


def test_regularized_chan_spectrum_matches_oracle(firm):
    N, order = 16, 2
    R, K32, Kf = _system(N, 5, 620)
    ker0 = float(K32[N, N, N])
    lam, mu = 1e-2 * ker0, 1e-3 * ker0
    plan = firm.Plan(N, R)
    plan.kernel_set(dev(K32))
    plan.set_regularizer(order, mu)
    t = plan.chan_spectrum(lam).cpu().numpy()
    ref = ofirm.chan_circulant_spectrum(Kf + mu * ofirm.regularizer_kernel(N, order), N, lam)
    assert rel(t, ref) < 1e-5


def test_regularized_solve_certified_by_oracle(firm):
    """CG and Chan PCG on the regularized system (lambda relative to Ker(0), FP64 refinement, FP64
    right-hand side and solution) reach 1e-6 under the oracle's FP64 operator."""
    N, order = 32, 1
    R, K32, Kf = _system(N, 3, 630)
    ker0 = float(K32[N, N, N])
    lam_rel, mu_rel = 1e-2, 1e-2
    plan = firm.Plan(N, R, precision=1, lambda_relative=1)
    plan.kernel_set(dev(K32))
    plan.set_regularizer(order, mu_rel)
    b = np.random.default_rng(7).standard_normal((N, N, N))
    T = ofirm.toeplitz_operator(Kf + mu_rel * ker0 * ofirm.regularizer_kernel(N, order))
    for pc in (None, torch.reciprocal(plan.chan_spectrum(lam_rel))):
        x, rep = plan.cg_solve(dev(b, torch.float64), lam_rel, 1e-6, 3000, precond=pc)
        xh = x.cpu().numpy().astype(np.float64)
        rr = np.linalg.norm(b - T(xh) - lam_rel * ker0 * xh) / np.linalg.norm(b)
        print(f"regularized {'PCG' if pc is not None else 'CG'}: {rep['iters']} iterations, oracle rel res {rr:.2e}",
              flush=True)
        assert rep["status"] == 0 and rr <= 1e-6 * 1.01
