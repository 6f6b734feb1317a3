"""GPU test of the gridding's view culling over more views than one group of block tests holds.

The spread tests the normal boxes of a work range's blocks of 512 views up to 512 blocks
(262,144 views) at a time, into a bit mask, then visits the live blocks.  A tile's work range
spans M / ceil(f M / 16384) views, f the fraction of planes that can meet the tile (the ratio of
its circumscribed radius to its distance from the centre), so the far tiles of the kernel grid
(4N, tile 13) get ranges of more than 262,144 views once N >= 128 and M > 262,144.  At N = 128
with M = 300,000 views, the kernel Ker (a sum over the views, the eq. kernel) of all the views
must equal the sum of the kernels of two plans that split the views (150,000 each, whose ranges
fit one group), to FP32 rounding.  The complex spread (A*b) runs the same culling code."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import rel, small_geometry  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def firm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1307_5824_amd import firm as f
    return f


def test_kernel_of_many_views_is_the_sum_over_a_split(firm):
    N, M, M1 = 128, 300_000, 150_000
    print(f"kernel over {M} views at N = {N}, against two plans of {M1} and {M - M1}", flush=True)
    R, sh, grp, table = small_geometry(N, M, 101, 3, True)
    kers = []
    for sel in (slice(0, M), slice(0, M1), slice(M1, M)):
        plan = firm.Plan(N, R[sel], shifts=sh[sel], ctf_group=grp[sel], ctf_table=table)
        plan.kernel_precompute()
        torch.cuda.synchronize()
        kers.append(plan.kernel_get().detach().cpu().numpy().astype(np.float64))
        plan.close()
    err = rel(kers[0], kers[1] + kers[2])
    print(f"  rel L2 {err:.2e}", flush=True)
    assert err < 2e-6
