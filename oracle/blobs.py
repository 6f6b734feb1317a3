"""Closed forms for Gaussian-blob volumes (test infrastructure only).

A blob volume is phi(x) = sum_b a_b exp(-||x - c_b||^2 / (2 s_b^2)) in voxel
units (grid spacing a = 1, section 3.1).  Its continuous Fourier transform with
the paper's convention (section 2.2, exp(-i <omega, x>)) is

    (F phi)(w) = sum_b a_b (2 pi s_b^2)^{3/2} exp(-s_b^2 ||w||^2 / 2) exp(-i <c_b, w>),

and its projection along x3 after rotation by R (section 3.1,
phi_R(x) = phi(R^{-1} x)) is a sum of 2D Gaussians centred at the first two
coordinates of R c_b with weight a_b sqrt(2 pi) s_b.

A blob with s_b = 0 is read as a point source a_b delta(x - c_b) whose transform
is a_b exp(-i <c_b, w>).
"""
import numpy as np

from . import firm


def sample_volume(N, centers, sigmas, amps):
    """V(n) = phi(n) on the N^3 grid n in [-N/2, N/2)^3 (section 3.1, volume sampling)."""
    n = firm.voxel_coords(N)
    g1, g2, g3 = np.meshgrid(n, n, n, indexing="ij")
    V = np.zeros((N, N, N))
    for c, s, a in zip(np.asarray(centers).reshape(-1, 3), np.ravel(sigmas), np.ravel(amps)):
        d2 = (g1 - c[0]) ** 2 + (g2 - c[1]) ** 2 + (g3 - c[2]) ** 2
        V += a * np.exp(-d2 / (2.0 * s * s))
    return V


def fourier_at(points, centers, sigmas, amps):
    """(F phi)(w) at points w (..., 3)."""
    w = np.asarray(points, dtype=np.float64)
    out = np.zeros(w.shape[:-1], dtype=np.complex128)
    w2 = np.sum(w * w, axis=-1)
    for c, s, a in zip(np.asarray(centers).reshape(-1, 3), np.ravel(sigmas), np.ravel(amps)):
        amp = a * (2.0 * np.pi * s * s) ** 1.5 * np.exp(-0.5 * s * s * w2) if s > 0 else a
        out += amp * np.exp(-1j * (w @ np.asarray(c, dtype=np.float64)))
    return out


def slices(N, rotations, centers, sigmas, amps, h=None, shifts=None):
    """Clean Fourier slices b(k, m) of translated, CTF-filtered projections of a blob volume:
    h_m(||omega_k||) exp(-i <omega_k, s_m>) (F phi)(xi_{k,m}).  By the projection-slice theorem
    (eq. continuous_fps) this is the 2D transform of the m-th image."""
    xi = firm.sample_points(N, rotations)
    b = fourier_at(xi, centers, sigmas, amps)
    if h is not None:
        b = b * h
    if shifts is not None:
        b = b * np.conj(firm.shift_phase(N, shifts))
    return b


def projection_image(N, R, centers, sigmas, amps, shift=None):
    """Real-space projection (P_R phi)(x1, x2) = integral of phi(R^{-1} x) dx3 on the pixel grid
    x in [-N/2, N/2)^2 (section 3.1), for blobs with s_b > 0.  With a shift s the image is that
    of a particle off-centre by s, J(x - s) (the images that section 3.1 re-shifts to their
    centres)."""
    x = firm.voxel_coords(N)
    g1, g2 = np.meshgrid(x, x, indexing="ij")
    img = np.zeros((N, N))
    R = np.asarray(R, dtype=np.float64).reshape(3, 3)
    sh = np.zeros(2) if shift is None else np.asarray(shift, dtype=np.float64).reshape(2)
    for c, s, a in zip(np.asarray(centers).reshape(-1, 3), np.ravel(sigmas), np.ravel(amps)):
        rc = R @ np.asarray(c, dtype=np.float64)
        d2 = (g1 - rc[0] - sh[0]) ** 2 + (g2 - rc[1] - sh[1]) ** 2
        img += a * np.sqrt(2.0 * np.pi) * s * np.exp(-d2 / (2.0 * s * s))
    return img


def centred_dft2(img, k1, k2):
    """2D DFT of an image on [-N/2, N/2)^2 at integer frequencies k (section 2.2 convention)."""
    N = img.shape[0]
    x = firm.voxel_coords(N)
    e1 = np.exp(-2j * np.pi * np.outer(k1, x) / N)
    e2 = np.exp(-2j * np.pi * np.outer(k2, x) / N)
    return np.einsum("ja,ab,jb->j", e1, img, e2)
