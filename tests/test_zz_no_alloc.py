"""The no-allocation variant of firm_precond_from_output, called through the C ABI, against the
allocating entry point on the same inputs: two calls in a row, the second on a smaller grid."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import pcnet as opc  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def firm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1307_5824_amd import firm as f
    return f


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _plan(firm, N, ker0):
    """A plan whose kernel is ker0 times a delta: Ker(0) = ker0 (the diagonal depends on the kernel
    only through Ker(0))."""
    plan = firm.Plan(N, [[1.0, 0, 0, 0, 1.0, 0, 0, 0, 1.0]])
    K = torch.zeros((2 * N,) * 3, device="cuda")
    K[N, N, N] = ker0
    plan.kernel_set(K)
    return plan


def test_noalloc_matches_allocating_entry_point(firm):
    lib = firm.lib
    rng = np.random.default_rng(77)
    for N, res, ker0 in ((128, 128, 3.0), (32, 32, 5.0)):   # the second call is smaller
        plan = _plan(firm, N, ker0)
        o = torch.as_tensor(rng.standard_normal((res,) * 3), dtype=torch.float32).cuda()
        t = torch.as_tensor(rng.uniform(0.5, 6.0, (N,) * 3), dtype=torch.float32).cuda()
        d_ref = torch.empty((N,) * 3, device="cuda")
        d = torch.full((N,) * 3, float("nan"), device="cuda")
        assert lib.firm_precond_from_output(plan.h, _ptr(o), res, _ptr(t), _ptr(d_ref)) == firm.FIRM_OK
        assert lib.firm_precond_from_output_noalloc(plan.h, _ptr(o), res, _ptr(t), _ptr(d)) == firm.FIRM_OK
        torch.cuda.synchronize()
        print(f"N={N} res={res}: max |d - d_ref| = {(d - d_ref).abs().max().item():.3e}", flush=True)
        assert torch.equal(d, d_ref)          # the same kernels on the same inputs
        ref = opc.diagonal(o.cpu().numpy().astype(np.float64), N, ker0, t.cpu().numpy().astype(np.float64))
        got = d.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)
        plan.close()


def test_noalloc_rejects_grids_beyond_the_scratch(firm):
    lib = firm.lib
    plan = _plan(firm, 32, 2.0)
    o = torch.zeros((256,) * 3, device="cuda")
    t = torch.ones((32,) * 3, device="cuda")
    d = torch.empty((32,) * 3, device="cuda")
    assert lib.firm_precond_from_output_noalloc(plan.h, _ptr(o), 256, _ptr(t), _ptr(d)) == firm.FIRM_ERR_ARG
    assert b"128" in lib.firm_last_error(plan.h)
    plan.close()
