"""Degenerate and boundary cases of the GPU path against the FP64 oracle.

* Axis-aligned views (the 24 rotations of the cube): every sample point lies on the fine grid
  and every cell on a tile boundary, the worst case of the tile enumeration.
* One view, and one view repeated: Ker is supported on one plane (the oracle pins the
  single-view kernel to a 2D sum), M copies scale it by M; enough copies to overflow the
  spread's view slots within one round.
* A zero right-hand side: every solver mode returns x = 0 at once.
Tolerances as in the parity tests (1e-5 relative L2 for FP32 operators).
"""
import itertools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import ker_to_centred, rel, small_geometry  # noqa: E402
from oracle import firm as ofirm  # noqa: E402
from paper_1307_5824_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-5


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
    return t.detach().cpu().numpy()


def cube_rotations():
    out = []
    for perm in itertools.permutations(range(3)):
        for sg in itertools.product([1.0, -1.0], repeat=3):
            R = np.zeros((3, 3))
            for i, j in enumerate(perm):
                R[i, j] = sg[i]
            if np.linalg.det(R) > 0:
                out.append(R)
    return np.array(out)


@pytest.mark.parametrize("N", [16, 32])
def test_axis_aligned_views(firm, N):
    """Kernel, back-projection and forward projection with all sample points on the grid."""
    print(f"axis-aligned views N={N}", flush=True)
    R = cube_rotations()
    M = R.shape[0]
    rng = np.random.default_rng(N)
    sh = rng.uniform(-2, 2, (M, 2))
    plan = firm.Plan(N, R, shifts=sh)
    plan.kernel_precompute()
    assert rel(host(plan.kernel_get()).astype(np.float64), ker_to_centred(ofirm.kernel_direct(N, R), N)) < TOL
    P = ofirm.slice_point_count(N)
    b = (rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))).astype(np.complex64)
    atb = host(plan.backproject(dev(b, torch.complex64))).astype(np.float64)
    ref = ofirm.back_project(ofirm.recentre(b.astype(np.complex128), N, sh), N, R).real
    assert rel(atb, ref) < TOL
    V = rng.standard_normal((N, N, N)).astype(np.float32)
    fv = host(plan.forward_project(dev(V))).astype(np.complex128)
    reff = ofirm.forward_project(V.astype(np.float64), R) * np.conj(ofirm.shift_phase(N, sh))
    assert rel(fv, reff) < TOL


def test_many_copies_of_one_view_fill_the_view_slots(firm):
    """700 copies of one view, each with one of three CTFs.  Every copy meets the same tiles,
    more than the spread's view slots of one round hold (512 for Ker, 256 for A*b), so the
    queues are processed and the slots reused in the middle of a round.  With one geometry the
    oracle sums reduce to one-view ones: Ker = sum over the groups of count * the one-view
    kernel with that CTF, A*b = the one-view back-projection of sum_m h_m b_m, and every slice
    of the forward projection is h_m times the one-view slice."""
    N, M, G = 16, 700, 3
    print(f"many copies of one view N={N} M={M}", flush=True)
    R1, _, _, _ = small_geometry(N, 1, 17)
    rng = np.random.default_rng(18)
    table = synth.ctf_table(N, synth.defoci(G, rng))
    grp = rng.integers(0, G, M).astype(np.int32)
    plan = firm.Plan(N, np.repeat(R1, M, axis=0), ctf_group=grp, ctf_table=table)
    plan.kernel_precompute()
    ker_ref = sum(np.count_nonzero(grp == g) * ofirm.kernel_direct(N, R1, ofirm.ctf_weights(N, 1, [g], table)).real
                  for g in range(G))
    assert rel(host(plan.kernel_get()).astype(np.float64), ker_to_centred(ker_ref, N)) < TOL
    P = ofirm.slice_point_count(N)
    h = ofirm.ctf_weights(N, M, grp, table)
    b = (rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))).astype(np.complex64)
    atb = host(plan.backproject(dev(b, torch.complex64))).astype(np.float64)
    atb_ref = ofirm.back_project((h * b.astype(np.complex128)).sum(axis=0, keepdims=True), N, R1).real
    assert rel(atb, atb_ref) < TOL
    V = rng.standard_normal((N, N, N)).astype(np.float32)
    fv = host(plan.forward_project(dev(V))).astype(np.complex128)
    assert rel(fv, h * ofirm.forward_project(V.astype(np.float64), R1)) < TOL


def test_single_and_repeated_view(firm):
    N = 16
    R1, _, _, _ = small_geometry(N, 1, 5)
    one = firm.Plan(N, R1)
    one.kernel_precompute()
    k1 = host(one.kernel_get()).astype(np.float64)
    assert rel(k1, ker_to_centred(ofirm.kernel_direct(N, R1), N)) < TOL
    five = firm.Plan(N, np.repeat(R1, 5, axis=0))
    five.kernel_precompute()
    assert rel(host(five.kernel_get()).astype(np.float64), 5 * k1) < TOL
    # one view leaves most of the volume unseen: CG on A*A + lambda still converges (FP64 output:
    # at this conditioning the FP32 rounding of x alone moves the residual to ~1e-5)
    atb = dev(np.random.default_rng(6).standard_normal((N, N, N)), torch.float64)
    plan = firm.Plan(N, R1, precision=1, lambda_relative=1)
    plan.kernel_precompute()
    _, rep = plan.cg_solve(atb, 1e-2, 1e-5, 3000)
    assert rep["status"] == 0 and rep["true_rel_res"] <= 1e-5 * (1 + 1e-6)


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("with_precond", [False, True])
def test_zero_right_hand_side(firm, precision, with_precond):
    if precision == 2 and with_precond:
        pytest.skip("precision 2 runs plain CG")
    N = 16
    R, _, _, _ = small_geometry(N, 20, 8)
    plan = firm.Plan(N, R, precision=precision, lambda_relative=1)
    plan.kernel_precompute()
    d = torch.ones((N, N, N), device="cuda") if with_precond else None
    x, rep = plan.cg_solve(torch.zeros((N, N, N), device="cuda"), 1e-2, 1e-5, 100, precond=d)
    assert rep["status"] == 0 and rep["iters"] == 0
    assert float(torch.abs(x).max()) == 0.0
