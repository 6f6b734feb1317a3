"""GPU tests of the fixed-point gridding's units (paper_1307_5824_amd/csrc/spread.hip): the LDS
tile holds 64-bit integer sums of terms rounded in units of 1/fxs, fxs a power of two set from the
largest possible term (for A*b from the largest |component| of the data, found on the device; for
Ker from the CTF table).  The results must follow the data's scale over many decades, be exactly
zero for zero data, and keep FP32-level accuracy when the data span a wide range of magnitudes.
Expected values come from the oracle (the plain sums of eq. backprojection and eq. kernel)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import ker_to_centred, rel, small_geometry  # noqa: E402
from oracle import firm as ofirm  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def firm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1307_5824_amd import firm as f
    return f


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def disk_radii(N):
    ks = [(k1, k2) for k1 in range(-N // 2, N // 2 + 1) for k2 in range(-N // 2, N // 2 + 1)
          if 4 * (k1 * k1 + k2 * k2) <= N * N]
    return np.hypot(*np.array(ks, dtype=np.float64).T)


@pytest.mark.parametrize("scale", [1e-20, 1.0, 1e20])
def test_backprojection_follows_the_data_scale(firm, scale):
    """A*(c b) = c A*b: the unit follows max|b|, so tiny and huge data keep their accuracy."""
    N, M = 16, 60
    print(f"backprojection scale {scale:g}", flush=True)
    R, sh, grp, table = small_geometry(N, M, 91, 3, True)
    rng = np.random.default_rng(92)
    P = ofirm.slice_point_count(N)
    b = (rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))) * scale
    b32 = b.astype(np.complex64)
    plan = firm.Plan(N, R, shifts=sh, ctf_group=grp, ctf_table=table)
    got = host(plan.backproject(torch.as_tensor(b32).cuda()))
    h = ofirm.ctf_weights(N, M, grp, table)
    ref = ofirm.back_project(ofirm.recentre(b32.astype(np.complex128), N, sh), N, R, h).real
    print(f"  rel L2 {rel(got, ref):.2e}", flush=True)
    assert rel(got, ref) < TOL
    plan.close()


def test_backprojection_of_zero_data_is_zero(firm):
    N, M = 16, 40
    R, sh, grp, table = small_geometry(N, M, 93, 2, True)
    plan = firm.Plan(N, R, shifts=sh, ctf_group=grp, ctf_table=table)
    b = torch.zeros((M, ofirm.slice_point_count(N)), dtype=torch.complex64, device="cuda")
    got = host(plan.backproject(b))
    assert np.all(got == 0.0)
    plan.close()


@pytest.mark.parametrize("power", [4.0, 8.0])
def test_backprojection_of_data_spanning_many_decades(firm, power):
    """Gaussian data under a radial envelope (1 + |k|/4)^-power: the components' magnitudes from the
    origin to the disk's edge (|k| = N/2) span (1 + N/8)^power, 625 and 3.9e5 at N = 32.  The unit
    is set by the largest, so the smallest terms enter with a few thousand units of resolution;
    the result must stay within the FP32 tolerance of the direct sums."""
    N, M = 32, 40
    print(f"backprojection envelope power {power}", flush=True)
    R, sh, grp, table = small_geometry(N, M, 94, 3, True)
    rng = np.random.default_rng(95)
    env = (1.0 + disk_radii(N) / 4.0) ** (-power)
    P = env.size
    b = (rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))) * env[None, :]
    b32 = b.astype(np.complex64)
    plan = firm.Plan(N, R, shifts=sh, ctf_group=grp, ctf_table=table)
    got = host(plan.backproject(torch.as_tensor(b32).cuda()))
    h = ofirm.ctf_weights(N, M, grp, table)
    ref = ofirm.back_project(ofirm.recentre(b32.astype(np.complex128), N, sh), N, R, h).real
    print(f"  rel L2 {rel(got, ref):.2e}", flush=True)
    assert rel(got, ref) < TOL
    plan.close()


@pytest.mark.parametrize("scale", [1e-8, 1e8])
def test_kernel_follows_the_ctf_scale(firm, scale):
    """Ker(c h) = c^2 Ker(h): the unit follows the CTF table's largest |h|."""
    N, M = 16, 80
    print(f"kernel CTF scale {scale:g}", flush=True)
    R, _, grp, table = small_geometry(N, M, 96, 3)
    table = (table * scale).astype(np.float32)
    plan = firm.Plan(N, R, ctf_group=grp, ctf_table=table)
    plan.kernel_precompute()
    got = host(plan.kernel_get())
    h = ofirm.ctf_weights(N, M, grp, table)
    ref = ker_to_centred(ofirm.kernel_direct(N, R, h), N)
    print(f"  rel L2 {rel(got, ref):.2e}", flush=True)
    assert rel(got, ref) < TOL
    plan.close()


@pytest.mark.parametrize("W,bound", [(4, 1e-2), (5, 1e-3), (6, 1e-4), (7, 1e-5), (8, 1e-5)])
def test_gridding_at_every_window_width(firm, W, bound):
    """Every window width the plan accepts runs its own lane map and tile (rows split among the
    lane groups, pitch, LDS size); Ker and A*b against the direct sums within a bound that the
    window's own error sets (measured: 6e-4, 7e-5, 7e-6, 8e-7 and 2e-7 for widths 4 .. 8)."""
    N, M = 16, 40
    print(f"window width {W}", flush=True)
    R, sh, grp, table = small_geometry(N, M, 97, 2, True)
    rng = np.random.default_rng(98)
    P = ofirm.slice_point_count(N)
    b32 = (rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))).astype(np.complex64)
    plan = firm.Plan(N, R, shifts=sh, ctf_group=grp, ctf_table=table, kb_width=W)
    plan.kernel_precompute()
    ker = host(plan.kernel_get())
    atb = host(plan.backproject(torch.as_tensor(b32).cuda()))
    h = ofirm.ctf_weights(N, M, grp, table)
    ker_ref = ker_to_centred(ofirm.kernel_direct(N, R, h), N)
    atb_ref = ofirm.back_project(ofirm.recentre(b32.astype(np.complex128), N, sh), N, R, h).real
    ek, ea = rel(ker, ker_ref), rel(atb, atb_ref)
    print(f"  Ker rel L2 {ek:.2e}, A*b rel L2 {ea:.2e}", flush=True)
    assert ek < bound and ea < bound
    plan.close()
