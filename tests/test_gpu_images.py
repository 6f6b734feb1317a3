"""GPU parity of Step 1 (section 3.4: images -> Fourier slices) and of the real-space image
generator against the FP64 oracle.

Expected values: oracle.blobs.centred_dft2 (the centred 2D DFT of section 2.2 at the disk
points) and oracle.blobs.projection_image (section 3.1 projections, translated images).
Tolerance 1e-5 relative L2: two FP32 FFT passes of length N (~1e-7 each); the image generator
evaluates FP32 Gaussians (~1e-7 relative) with a cutoff at 9 sigma (exp(-40.5)).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import rel, small_geometry  # noqa: E402
from oracle import blobs as oblobs  # noqa: E402
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


def _blobs(rng, B, N, spread=0.2):
    c = rng.uniform(-spread * N, spread * N, size=(B, 3))
    s = rng.uniform(1.5, 2.5, size=B)
    a = rng.uniform(0.5, 1.0, size=B)
    return c, s, a


@pytest.mark.parametrize("N,M", [(8, 5), (16, 30), (64, 3)])
def test_images_to_slices_matches_oracle(firm, N, M):
    """Every disk value of white-noise images (all frequencies present) vs the direct DFT."""
    print(f"images_to_slices N={N} M={M}", flush=True)
    R, _, _, _ = small_geometry(N, M, 60 + N)
    img = np.random.default_rng(N).standard_normal((M, N, N)).astype(np.float32)
    plan = firm.Plan(N, R)
    got = host(plan.images_to_slices(dev(img))).astype(np.complex128)
    k1, k2 = ofirm.disk_points(N)
    ref = np.stack([oblobs.centred_dft2(img[m].astype(np.float64), k1, k2) for m in range(M)])
    assert rel(got, ref) < TOL


def test_images_to_slices_full_size_sampled(firm):
    """N = 256, 4,000 images (two batches of the 1 GiB workspace): 96 sampled disk values of
    four images, among them the boundary points and images of both batches."""
    N, M = 256, 4000
    print(f"images_to_slices full size N={N} M={M}", flush=True)
    R = synth.haar_rotations(M, np.random.default_rng(8))
    plan = firm.Plan(N, R)
    g = torch.Generator(device="cuda").manual_seed(9)
    img = torch.randn((M, N, N), device="cuda", generator=g)
    b = plan.images_to_slices(img)
    k1, k2 = ofirm.disk_points(N)
    edge = np.flatnonzero((np.abs(k1) == N // 2) | (np.abs(k2) == N // 2))
    pick = np.concatenate([edge, np.random.default_rng(10).integers(0, plan.P, 20)])
    for m in (0, 1, 3700, M - 1):
        got = host(b[m, torch.as_tensor(pick).cuda()]).astype(np.complex128)
        ref = oblobs.centred_dft2(host(img[m]).astype(np.float64), k1[pick], k2[pick])
        assert rel(got, ref) < TOL, m


def test_synth_images_match_oracle(firm):
    """Translated projection images of a blob volume vs the oracle's real-space projection."""
    N, M, B = 32, 6, 5
    R, sh, _, _ = small_geometry(N, M, 70, 0, True)
    rng = np.random.default_rng(71)
    c, s, a = _blobs(rng, B, N)
    plan = firm.Plan(N, R, shifts=sh)
    got = host(plan.synth_images(c, s, a)).astype(np.float64)
    ref = np.stack([oblobs.projection_image(N, R[m], c, s, a, shift=sh[m]) for m in range(M)])
    assert rel(got, ref) < TOL


def test_synth_images_noise_statistics(firm):
    """Pixel noise: zero mean, variance = mean clean power / SNR, independent of the image."""
    N, M, B = 32, 40, 4
    R, sh, _, _ = small_geometry(N, M, 72, 0, True)
    c, s, a = _blobs(np.random.default_rng(73), B, N)
    plan = firm.Plan(N, R, shifts=sh)
    clean = host(plan.synth_images(c, s, a, seed=4)).astype(np.float64)
    noisy = host(plan.synth_images(c, s, a, snr=0.5, seed=4)).astype(np.float64)
    z = noisy - clean
    var = np.mean(clean ** 2) / 0.5
    n = z.size
    assert abs(z.mean()) < 5 * np.sqrt(var / n)
    assert abs(z.var() / var - 1) < 5 * np.sqrt(2.0 / n)
    assert abs(np.corrcoef(z.ravel(), clean.ravel())[0, 1]) < 5 / np.sqrt(n)


def test_images_pipeline_matches_fourier_generator(firm):
    """Real-space images -> Step 1 -> slices agree with the Fourier-space slice generator
    (projection-slice theorem, eq. continuous_fps) up to the pixel-sampling aliasing floor."""
    N, M, B = 64, 8, 5
    R, sh, _, _ = small_geometry(N, M, 74, 0, True)
    # blobs well inside the field of view, so that the images hold their whole projections
    c, s, a = _blobs(np.random.default_rng(75), B, N, spread=1 / 16)
    plan = firm.Plan(N, R, shifts=sh)
    b_img = host(plan.images_to_slices(plan.synth_images(c, s, a))).astype(np.complex128)
    b_fou = host(plan.synth_slices(c, s, a)).astype(np.complex128)
    assert rel(b_img, b_fou) < 1e-3
