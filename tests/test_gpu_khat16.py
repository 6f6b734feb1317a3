"""The 16-bit kernel spectrum (option khat_bf16: BF16 codes with a per-shell offset and scale).

Bar: the product with the 16-bit spectrum is within 1e-3 (relative L2) of the oracle's FP64
Toeplitz product, for kernels of view sets and CTFs like the workloads' (the encoding's error
is ~2^-9 of each shell's spread around its mean; measured ~6e-4 on such kernels); with FP64
iterative refinement (precision 1), where the FP64 residual uses the FP32 kernel, solves reach
the same 1e-5 true residual as with the FP32 spectrum.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import ker_to_centred, rel  # noqa: E402
from oracle import firm as ofirm  # noqa: E402
from paper_1307_5824_amd import synth  # noqa: E402

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


def _physical(N, M, seed):
    rng = np.random.default_rng(seed)
    R = synth.mixed_rotations(M, 10.0, 0.1, rng)
    table = synth.ctf_table(N, synth.defoci(6, rng))
    grp = rng.integers(0, 6, M).astype(np.int32)
    Ker = ofirm.kernel_direct(N, R, ofirm.ctf_weights(N, M, grp, table)).real
    return R, grp, table, Ker


@pytest.mark.parametrize("N,M,mode", [(16, 120, 1), (32, 60, 1), (32, 60, 2)])
def test_bf16_spectrum_product_within_1e3(firm, N, M, mode):
    print(f"khat16 apply N={N} M={M} mode={mode}", flush=True)
    R, grp, table, Ker = _physical(N, M, 500 + N)
    lam = 1e-2 * Ker[N - 1, N - 1, N - 1]
    x = np.random.default_rng(N).standard_normal((N, N, N))
    ref = ofirm.toeplitz_apply_fft(Ker, x).real + lam * x
    K = dev(ker_to_centred(Ker, N))
    p16 = firm.Plan(N, R, ctf_group=grp, ctf_table=table, khat_bf16=mode)
    p32 = firm.Plan(N, R, ctf_group=grp, ctf_table=table)
    p16.kernel_set(K)
    p32.kernel_set(K)
    e16 = rel(host(p16.apply_AtA(dev(x), lam)), ref)
    e32 = rel(host(p32.apply_AtA(dev(x), lam)), ref)
    print(f"product error: 16-bit spectrum {e16:.2e}, FP32 spectrum {e32:.2e}", flush=True)
    assert e16 < 1e-3
    assert e32 < 1e-5 and e16 > e32                       # the 16-bit copy is what was used


def test_bf16_spectrum_refined_solve(firm):
    """precision 1: 16-bit inner product, FP64 outer residual with the FP32 kernel.  The
    right-hand side is FP64, so the solve returns its FP64 iterate, the one the outer residual
    test stops on (an FP32 copy of it can exceed the tolerance by its own rounding)."""
    N, M = 32, 200
    R, grp, table, Ker = _physical(N, M, 77)
    K = dev(ker_to_centred(Ker, N))
    atb = dev(np.random.default_rng(3).standard_normal((N, N, N)), torch.float64)
    sols = {}
    for bf in (0, 1):
        plan = firm.Plan(N, R, ctf_group=grp, ctf_table=table, precision=1, lambda_relative=1, khat_bf16=bf)
        plan.kernel_set(K)
        x, rep = plan.cg_solve(atb, 1e-2, 1e-5, 3000)
        print(f"khat_bf16={bf}: {rep['iters']} iterations, true residual {rep['true_rel_res']:.2e}", flush=True)
        assert rep["status"] == 0 and rep["true_rel_res"] <= 1e-5 * (1 + 1e-6)
        sols[bf] = host(x)
    assert rel(sols[1], sols[0]) < 1e-4
