"""Shared helpers of the GPU parity tests: inputs from the seeded generators, expected values
from the oracle only."""
import numpy as np

from oracle import firm as ofirm
from paper_1307_5824_amd import synth


def rel(a, b):
    """Relative L2 distance ||a - b|| / ||b||, complex-aware."""
    cplx = np.iscomplexobj(a) or np.iscomplexobj(b)
    a = np.asarray(a, dtype=np.complex128 if cplx else np.float64)
    b = np.asarray(b, dtype=np.complex128 if cplx else np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def ker_to_centred(Ker, N):
    """Oracle (2N-1)^3 kernel (offsets -N+1..N-1) -> the library's (2N)^3 centred layout
    (index j = offset + N; j = 0 planes zero)."""
    out = np.zeros((2 * N,) * 3, dtype=np.float64)
    out[1:, 1:, 1:] = np.real(Ker)
    return out


def small_geometry(N, M, seed, groups=0, shifts=False):
    rng = np.random.default_rng(seed)
    R = synth.haar_rotations(M, rng)
    table = grp = sh = None
    if groups:
        table = synth.ctf_table(N, synth.defoci(groups, rng))
        grp = rng.integers(0, groups, M).astype(np.int32)
    if shifts:
        sh = rng.uniform(-2, 2, size=(M, 2))
    return R, sh, grp, table


def even_random_kernel(N, rng):
    """A real, even Toeplitz kernel on offsets (-N, N)^3 (oracle-side input for product tests)."""
    K = rng.standard_normal((2 * N - 1,) * 3)
    return 0.5 * (K + K[::-1, ::-1, ::-1])


def gaussian_kernel(N, width, cos_amp=0.1):
    """Real, even, smooth kernel exp(-|n|^2 / (2 w^2)) + cos_amp cos(pi n1 / N) on offsets (-N, N)^3."""
    n = np.arange(-N + 1, N, dtype=np.float64)
    g = np.exp(-n * n / (2 * width * width))
    K = g[:, None, None] * g[None, :, None] * g[None, None, :]
    K += cos_amp * np.cos(np.pi * n / N)[:, None, None] * np.ones((1, 2 * N - 1, 2 * N - 1))
    return K


__all__ = ["rel", "ker_to_centred", "small_geometry", "even_random_kernel", "gaussian_kernel", "ofirm"]
