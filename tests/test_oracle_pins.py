"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics, not by itself.

Each test names the passage or identity it checks.  None of them runs on a GPU.
"""
import math
import os

import numpy as np
import pytest

from oracle import blobs, direct, firm
from paper_1307_5824_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


def _load_golden_pairs(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append([int(t) for t in line.split()])
    return rows


# ------------------------------------------------ truncation disk (eq. truncation) --

def test_disk_counts_match_gauss_circle_table():
    """P(N) = number of lattice points with ||k|| <= N/2: the Gauss circle counts
    (OEIS A000328) stored in tests/golden/gauss_circle.txt."""
    for r, count in _load_golden_pairs("gauss_circle.txt"):
        assert firm.slice_point_count(2 * r) == count


@pytest.mark.parametrize("N", [8, 16, 32, 64, 128, 256])
def test_disk_counts_by_row_formula(N):
    """Independent count: row k1 holds 2 floor(sqrt(N^2/4 - k1^2)) + 1 points."""
    r2 = N * N // 4
    count = sum(2 * math.isqrt(r2 - k1 * k1) + 1 for k1 in range(-N // 2, N // 2 + 1))
    assert firm.slice_point_count(N) == count
    assert direct.slice_points(N) == count


def test_disk_order_symmetric():
    """The canonical order lists -k at index P-1-j; the four boundary points ||k|| = N/2 are kept."""
    for N in (8, 16, 32):
        k1, k2 = firm.disk_points(N)
        assert np.array_equal(k1[::-1], -k1) and np.array_equal(k2[::-1], -k2)
        on_edge = (4 * (k1 ** 2 + k2 ** 2) == N * N).sum()
        assert on_edge == 4 * (1 if N % 2 == 0 else 0) + 4 * sum(
            1 for a in range(1, N // 2) if math.isqrt(N * N // 4 - a * a) ** 2 == N * N // 4 - a * a)


# ------------------------------------------------ adjoint (section 3.2) --

@pytest.mark.parametrize("N,M", [(8, 5), (16, 3)])
def test_adjoint_identity(N, M):
    """<A V, g> = <V, A* g> with <a, b> = sum a conj(b) (section 2.1 and the definition of A*)."""
    rng = _rng(1)
    R = synth.haar_rotations(M, rng)
    table = synth.ctf_table(N, [1.5e4, 2.5e4])
    grp = rng.integers(0, 2, M)
    h = firm.ctf_weights(N, M, grp, table)
    V = rng.standard_normal((N, N, N)) + 1j * rng.standard_normal((N, N, N))
    P = firm.slice_point_count(N)
    g = rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))
    lhs = np.vdot(g, firm.forward_project(V, R, h))            # sum A(V) conj(g)
    rhs = np.vdot(firm.back_project(g, N, R, h), V)           # sum V conj(A* g)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_forward_projector_plain_sum():
    """A at a few points against a triple Python loop over voxels (eq. forward-projector)."""
    rng = _rng(2)
    N, M = 8, 2
    R = synth.haar_rotations(M, rng)
    V = rng.standard_normal((N, N, N))
    b = firm.forward_project(V, R)
    k1, k2 = firm.disk_points(N)
    for m, j in [(0, 3), (1, 20), (1, 48)]:
        om = np.array([2 * np.pi * k1[j] / N, 2 * np.pi * k2[j] / N, 0.0])
        xi = np.linalg.solve(R[m], om)
        s = 0j
        for i1 in range(N):
            for i2 in range(N):
                for i3 in range(N):
                    n = np.array([i1, i2, i3]) - N // 2
                    s += V[i1, i2, i3] * np.exp(-1j * n @ xi)
        assert abs(s - b[m, j]) <= 1e-12 * max(1.0, abs(s))


# ------------------------------------------------ projection-slice theorem (section 3.1) --

def _small_blobs(rng, B=3, N=32):
    c = rng.uniform(-3, 3, size=(B, 3))
    s = rng.uniform(1.5, 2.5, size=B)
    a = rng.uniform(0.5, 1.0, size=B)
    return c, s, a


def test_projection_slice_blobs_fourier():
    """A(V_blob)(k, m) equals the closed-form transform of the blob at xi_{k,m} up to the aliasing
    floor exp(-s^2 pi^2 / 2) ~ 1.5e-5 of sampling (eq. continuous_fps and its discrete form)."""
    rng = _rng(3)
    N, M = 32, 3
    c, s, a = _small_blobs(rng)
    R = synth.haar_rotations(M, rng)
    V = blobs.sample_volume(N, c, s, a)
    b = firm.forward_project(V, R)
    ref = blobs.slices(N, R, c, s, a)
    err = np.linalg.norm(b - ref) / np.linalg.norm(ref)
    assert err < 1e-3


def test_projection_slice_blobs_real_space():
    """The centred 2D DFT of the real-space projection image (section 3.1: integral of
    phi(R^{-1} x) along x3) equals the slice A(V)(., m): fixes the sign, 2 pi, R vs R^{-1}
    and centring conventions independently of the Fourier-side closed form."""
    rng = _rng(4)
    N, M = 32, 2
    c, s, a = _small_blobs(rng)
    R = synth.haar_rotations(M, rng)
    V = blobs.sample_volume(N, c, s, a)
    b = firm.forward_project(V, R)
    k1, k2 = firm.disk_points(N)
    for m in range(M):
        img = blobs.projection_image(N, R[m], c, s, a)
        f = blobs.centred_dft2(img, k1, k2)
        assert np.linalg.norm(f - b[m]) / np.linalg.norm(f) < 1e-3


def test_shifted_projection_image_matches_fourier_closed_form():
    """The image of a particle off-centre by s (real space, J(x - s)) has the centred DFT
    exp(-i <omega, s>) times the unshifted slice: the real-space generator's shift sign agrees
    with the Fourier closed form's, up to the sampling-aliasing floor."""
    rng = _rng(11)
    N = 32
    c, s, a = _small_blobs(rng)
    R = synth.haar_rotations(1, rng)
    sh = np.array([1.7, -2.3])
    k1, k2 = firm.disk_points(N)
    img = blobs.projection_image(N, R[0], c, s, a, shift=sh)
    f = blobs.centred_dft2(img, k1, k2)
    ref = blobs.slices(N, R, c, s, a, shifts=sh[None, :])[0]
    assert np.linalg.norm(f - ref) / np.linalg.norm(ref) < 1e-3
    f0 = blobs.centred_dft2(blobs.projection_image(N, R[0], c, s, a), k1, k2)
    assert np.linalg.norm(f - ref) < 0.1 * np.linalg.norm(f0 - ref)   # the shift matters


def test_centred_dft2_is_shifted_fft2():
    """The centred DFT at integer frequencies is numpy's FFT of the image with its centre moved
    to index 0, read at k mod N; the boundary k_d = +N/2 takes the value of -N/2."""
    N = 16
    img = np.random.default_rng(12).standard_normal((N, N))
    k1, k2 = firm.disk_points(N)
    f = blobs.centred_dft2(img, k1, k2)
    F = np.fft.fft2(np.fft.ifftshift(img))
    assert np.max(np.abs(f - F[k1 % N, k2 % N])) < 1e-11 * np.max(np.abs(F))
    edge = (np.abs(k1) == N // 2) | (np.abs(k2) == N // 2)
    assert edge.sum() == 4


def test_c_blob_slices_match_numpy():
    """The plain-C closed form equals the numpy closed form, with CTF and shifts."""
    rng = _rng(5)
    N, M = 16, 4
    c, s, a = _small_blobs(rng, B=4, N=N)
    s[0] = 0.0                                       # one point source
    R = synth.haar_rotations(M, rng)
    table = synth.ctf_table(N, [1.2e4, 2.8e4])
    grp = rng.integers(0, 2, M).astype(np.int32)
    sh = rng.uniform(-2, 2, size=(M, 2))
    h = firm.ctf_weights(N, M, grp, table)
    ref = blobs.slices(N, R, c, s, a, h=h, shifts=sh)
    got = direct.blob_slices(N, R, c, s, a, grp, table, sh)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


# ------------------------------------------------ Ker and the Toeplitz identity (section 3.2) --

@pytest.mark.parametrize("N,M", [(8, 6), (16, 2)])
def test_AstarA_equals_kernel_convolution(N, M):
    """A*(A x) = Ker * x by brute-force convolution (eq. toeplitz, toep2, property)."""
    rng = _rng(6)
    R = synth.haar_rotations(M, rng)
    table = synth.ctf_table(N, [2.0e4])
    h = firm.ctf_weights(N, M, np.zeros(M, int), table)
    x = rng.standard_normal((N, N, N))
    lhs = firm.back_project(firm.forward_project(x, R, h), N, R, h)
    Ker = firm.kernel_direct(N, R, h)
    rhs = firm.toeplitz_apply_brute(Ker, x)
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(lhs)


@pytest.mark.parametrize("N", [8, 16])
def test_embedding_matches_brute(N):
    """The 2N circulant embedding with zero wrap planes reproduces the Toeplitz product
    (eq. embedding_circulant, embedding_index, circ1)."""
    rng = _rng(7)
    R = synth.haar_rotations(3, rng)
    Ker = firm.kernel_direct(N, R)
    x = rng.standard_normal((N, N, N))
    a = firm.toeplitz_apply_brute(Ker, x)
    b = firm.toeplitz_apply_fft(Ker, x)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)


@pytest.mark.parametrize("N", [8, 16])
def test_real_toeplitz_operator_matches_embedding(N):
    """The real-FFT form with a precomputed spectrum equals the complex embedding product and the
    brute-force convolution for a real even kernel."""
    rng = _rng(21 + N)
    K = rng.standard_normal((2 * N - 1,) * 3)
    K = 0.5 * (K + K[::-1, ::-1, ::-1])
    x = rng.standard_normal((N, N, N))
    op = firm.toeplitz_operator(K, workers=2)
    ref = firm.toeplitz_apply_fft(K, x).real
    assert np.max(np.abs(op(x) - ref)) <= 1e-12 * np.max(np.abs(ref))
    if N == 8:
        assert np.max(np.abs(op(x) - firm.toeplitz_apply_brute(K, x))) <= 1e-11 * np.max(np.abs(ref))


def test_embedding_wrap_value_is_free():
    """Any value in the wrap slot gives the same cropped product (the reading of the
    embedding index map at i = N + 1)."""
    rng = _rng(8)
    N = 8
    Ker = firm.kernel_direct(N, synth.haar_rotations(2, rng))
    x = rng.standard_normal((N, N, N))
    c = firm.circulant_first_column(Ker, N)
    c2 = c.copy()
    c2[N, :, :] = rng.standard_normal((2 * N, 2 * N))
    c2[:, N, :] += 3.0
    xp = np.zeros((2 * N,) * 3)
    xp[:N, :N, :N] = x
    y1 = np.fft.ifftn(np.fft.fftn(c) * np.fft.fftn(xp))[:N, :N, :N]
    y2 = np.fft.ifftn(np.fft.fftn(c2) * np.fft.fftn(xp))[:N, :N, :N]
    assert np.linalg.norm(y1 - y2) <= 1e-12 * np.linalg.norm(y1)


def test_kernel_special_cases():
    """Ker(0) = sum of h^2; Ker is real and even (the disk is symmetric and h depends on ||k||
    only, refining Ker(-n) = conj Ker(n)); |Ker(n)| <= Ker(0)."""
    rng = _rng(9)
    N, M = 8, 7
    R = synth.haar_rotations(M, rng)
    table = synth.ctf_table(N, [1.1e4, 2.9e4])
    grp = rng.integers(0, 2, M)
    h = firm.ctf_weights(N, M, grp, table)
    Ker = firm.kernel_direct(N, R, h)
    c = N - 1
    assert abs(Ker[c, c, c] - np.sum(h * h)) <= 1e-12 * np.sum(h * h)
    assert np.max(np.abs(Ker.imag)) <= 1e-11 * Ker[c, c, c].real
    assert np.max(np.abs(Ker - Ker[::-1, ::-1, ::-1])) <= 1e-11 * Ker[c, c, c].real
    assert np.max(np.abs(Ker)) <= Ker[c, c, c].real * (1 + 1e-12)


def test_kernel_single_view_is_2d_sum():
    """R = I, h = 1: Ker(n) = sum_k cos(2 pi (n1 k1 + n2 k2) / N), independent of n3
    (brute-force double loop over the disk)."""
    N = 8
    Ker = firm.kernel_direct(N, np.eye(3)[None])
    for n1 in range(-N + 1, N):
        for n2 in range(-N + 1, N):
            s = 0.0
            for k1 in range(-N // 2, N // 2 + 1):
                for k2 in range(-N // 2, N // 2 + 1):
                    if 4 * (k1 * k1 + k2 * k2) <= N * N:
                        s += math.cos(2 * math.pi * (n1 * k1 + n2 * k2) / N)
            col = Ker[n1 + N - 1, n2 + N - 1, :]
            assert np.max(np.abs(col - s)) <= 1e-10 * 64


def test_kernel_axis_permutation_view_integer_points():
    """A view whose rotation is a signed axis permutation puts every sample on integer
    multiples of 2 pi / N; then Ker is N-periodic along the in-plane axes."""
    N = 8
    R = np.array([[[0, 0, 1], [1, 0, 0], [0, 1, 0]]], dtype=float)
    Ker = firm.kernel_direct(N, R)
    # xi = omega_1 (row 1) + omega_2 (row 2) = (omega_2, 0, omega_1): Ker depends on n1 and n3
    # through exp(2 pi i (n1 k2 + n3 k1) / N), so it is N-periodic in n1, n3 and constant in n2
    o = N - 1
    v1 = Ker[1 + o, 2 + o, 3 + o]
    assert abs(v1 - Ker[1 + o, 2 + o, 3 - N + o]) <= 1e-10 * 50
    assert abs(v1 - Ker[1 - N + o, 2 + o, 3 + o]) <= 1e-10 * 50
    assert np.max(np.abs(Ker[1 + o, :, 3 + o] - v1)) <= 1e-10 * 50


def test_c_direct_sums_match_numpy():
    """The plain-C direct sums of Ker and A* agree with the numpy oracle (two codings)."""
    rng = _rng(10)
    N, M = 16, 5
    R = synth.haar_rotations(M, rng)
    table = synth.ctf_table(N, [1.5e4, 2.2e4, 2.7e4])
    grp = rng.integers(0, 3, M).astype(np.int32)
    h = firm.ctf_weights(N, M, grp, table)
    offs = rng.integers(-N + 1, N, size=(6, 3))
    got = direct.kernel_at(offs, N, R, grp, table)
    ref = firm.kernel_at(offs, N, R, h)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.sum(h * h)
    P = firm.slice_point_count(N)
    b = (rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))).astype(np.complex64)
    sh = rng.uniform(-2, 2, size=(M, 2))
    vox = rng.integers(-N // 2, N // 2, size=(6, 3))
    got = direct.backproject_at(vox, b, N, R, grp, table, sh)
    g = firm.recentre(b.astype(np.complex128), N, sh)
    ref = firm.back_project_at(vox, g, N, R, h)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.sum(np.abs(b))


def test_shift_leaves_AstarA_unchanged():
    """Re-centring is a unit-modulus diagonal, so A*A (hence Ker) does not depend on shifts:
    back-projecting re-centred slices of a translated volume equals back-projecting the centred one."""
    rng = _rng(11)
    N, M = 8, 4
    R = synth.haar_rotations(M, rng)
    x = rng.standard_normal((N, N, N))
    sh = rng.uniform(-2, 2, size=(M, 2))
    b = firm.forward_project(x, R) * np.conj(firm.shift_phase(N, sh))
    lhs = firm.back_project(firm.recentre(b, N, sh), N, R)
    rhs = firm.back_project(firm.forward_project(x, R), N, R)
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(rhs)


# ------------------------------------------------ CG (section 3.3) --

def _system(N=8, M=6, lam=1e2, seed=12):
    rng = _rng(seed)
    R = synth.haar_rotations(M, rng)
    Ker = firm.kernel_direct(N, R)
    b = rng.standard_normal((N, N, N))

    def apply(v):
        return firm.toeplitz_apply_fft(Ker, v).real + lam * v
    return Ker, apply, b, lam


def test_cg_converges_to_dense_solve():
    """CG to 1e-13 equals a Cholesky solve of the dense (Ker(n - l) + lambda I) system."""
    N = 8
    Ker, apply, b, lam = _system(N)
    T = firm.toeplitz_dense(Ker, N).real + lam * np.eye(N ** 3)
    L = np.linalg.cholesky(T)
    xd = np.linalg.solve(L.T, np.linalg.solve(L, b.reshape(-1))).reshape(N, N, N)
    x = firm.cg(apply, b, tol=1e-13, iters=2000)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


def test_cg_iterates_are_krylov_minimisers():
    """CG's k-th iterate minimises the energy-norm error over K_k(T, b) (the Krylov definition)."""
    Ker, apply, b, lam = _system(8, lam=5e2)
    _, hist, _ = firm.cg(apply, b, iters=8, record=True)
    for k in (1, 3, 8):
        xk = firm.krylov_iterate(apply, b, k)
        assert np.linalg.norm(hist[k] - xk) <= 1e-8 * np.linalg.norm(xk)


def test_cg_energy_error_monotone():
    N = 8
    Ker, apply, b, lam = _system(N, lam=10.0)
    T = firm.toeplitz_dense(Ker, N).real + lam * np.eye(N ** 3)
    xs = np.linalg.solve(T, b.reshape(-1))
    _, hist, _ = firm.cg(apply, b, iters=25, record=True)
    e = [float((xs - h.reshape(-1)) @ T @ (xs - h.reshape(-1))) for h in hist]
    assert all(e[i + 1] <= e[i] * (1 + 1e-9) for i in range(len(e) - 1))


def test_tikhonov_limit():
    """lambda >> ||Ker||: x -> A*b / lambda; the solution varies continuously with lambda."""
    N = 8
    Ker, _, b, _ = _system(N)
    big = 1e8 * float(np.abs(Ker).sum())

    def apply(v):
        return firm.toeplitz_apply_fft(Ker, v).real + big * v
    x = firm.cg(apply, b, tol=1e-14, iters=50)
    assert np.linalg.norm(x - b / big) <= 1e-6 * np.linalg.norm(b / big)


def test_pcg_identity_preconditioner_equals_cg():
    """d = 1 gives the CG iterates."""
    Ker, apply, b, lam = _system(8, lam=1.0)
    _, h1, _ = firm.cg(apply, b, iters=12, record=True)
    _, h2, _ = firm.pcg(apply, firm.fourier_diagonal_precond(np.ones((8, 8, 8))), b, iters=12, record=True)
    for a, c in zip(h1, h2):
        assert np.linalg.norm(a - c) <= 1e-9 * max(1e-30, np.linalg.norm(a)) + 1e-300


def test_pcg_exact_inverse_one_step():
    """On a circulant operator with spectrum s(q) > 0, d = 1/s solves in one PCG step."""
    rng = _rng(13)
    N = 8
    s = np.fft.fftshift(rng.uniform(0.5, 5.0, (N, N, N)))
    s = 0.5 * (s + np.roll(s[::-1, ::-1, ::-1], 1, axis=(0, 1, 2)))   # s(q) = s(-q) in centred order
    sc = np.fft.ifftshift(s)

    def apply(v):
        return np.fft.ifftn(sc * np.fft.fftn(v)).real
    b = rng.standard_normal((N, N, N))
    x = firm.pcg(apply, firm.fourier_diagonal_precond(1.0 / s), b, iters=1)
    assert np.linalg.norm(apply(x) - b) <= 1e-12 * np.linalg.norm(b)


def test_chan_circulant_is_frobenius_projection():
    """T. Chan's optimal circulant equals the Frobenius-nearest circulant of the dense Toeplitz
    matrix: each wrapped diagonal averaged, then diagonalised by the DFT."""
    rng = _rng(14)
    N = 4
    Ker = firm.kernel_direct(N, synth.haar_rotations(3, rng))
    T = firm.toeplitz_dense(Ker, N).real
    idx = np.indices((N, N, N)).reshape(3, -1).T
    c = np.zeros((N, N, N))
    for j in np.ndindex(N, N, N):
        tot = 0.0
        for a in range(N ** 3):
            i = idx[a]
            l = (i - np.array(j)) % N
            tot += T[a, l[0] * N * N + l[1] * N + l[2]]
        c[j] = tot / N ** 3
    ref = np.fft.fftshift(np.fft.fftn(c).real)
    got = firm.chan_circulant_spectrum(Ker, N)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_chan_spectrum_is_fourier_diagonal_of_toeplitz():
    """The Chan spectrum is the diagonal of F T F^H / n (unitary DFT of the dense Toeplitz
    matrix): the Fourier diagonal used as the target of the learned preconditioner."""
    rng = _rng(15)
    N = 4
    Ker = firm.kernel_direct(N, synth.haar_rotations(4, rng)).real
    T = firm.toeplitz_dense(Ker, N)
    k = np.arange(N)
    F1 = np.exp(-2j * np.pi * np.outer(k, k) / N)
    F = np.kron(np.kron(F1, F1), F1)
    diag = np.real(np.einsum('ij,jk,ik->i', F, T, F.conj())) / N ** 3
    ref = np.fft.fftshift(diag.reshape(N, N, N))
    got = firm.chan_circulant_spectrum(Ker, N)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


# ------------------------------------------------ FSC (section 4) --

def test_fsc_properties():
    rng = _rng(15)
    V = rng.standard_normal((16, 16, 16))
    assert np.allclose(firm.fsc(V, V), 1.0)
    assert np.allclose(firm.fsc(V, 3.0 * V), 1.0)
    assert np.allclose(firm.fsc(V, -V), -1.0)
    W = rng.standard_normal((16, 16, 16))
    assert np.all(np.abs(firm.fsc(V, W)) < 0.6)


# ------------------------------------------------ noise and data --

def test_hermitian_noise_symmetry_and_power():
    rng = _rng(16)
    N, M = 16, 200
    P = firm.slice_point_count(N)
    n = firm.hermitian_noise(N, M, rng.standard_normal((M, P, 2)), 2.0)
    assert np.allclose(n[:, ::-1], np.conj(n))
    assert abs(np.mean(np.abs(n) ** 2) - 4.0) < 0.1


def test_backprojection_of_hermitian_data_is_real():
    """Slices of a real volume satisfy b(-k) = conj b(k); their back-projection is real."""
    rng = _rng(17)
    N, M = 8, 3
    R = synth.haar_rotations(M, rng)
    b = firm.forward_project(rng.standard_normal((N, N, N)), R)
    assert np.allclose(b[:, ::-1], np.conj(b))
    v = firm.back_project(b, N, R)
    assert np.max(np.abs(v.imag)) <= 1e-10 * np.max(np.abs(v.real))


def test_electron_wavelength_matches_paper_figure():
    """Fig. 2 of the paper quotes 2.51 pm, the relativistic wavelength at 200 kV."""
    assert abs(synth.electron_wavelength(200.0) * 100.0 - 2.51) < 0.005


# ------------------------------------- sampled direct sums against the full arrays --

@pytest.mark.parametrize("N,M", [(8, 4), (16, 3)])
def test_kernel_at_matches_full_kernel(N, M):
    """The sampled direct sums of eq. kernel (numpy and C) equal the full-array Ker, which is
    itself pinned by A*(A x) = Ker * x.  Offsets cover the corners (+-(N-1)) and mixed signs."""
    rng = _rng(30 + N)
    R = synth.haar_rotations(M, rng)
    table = synth.ctf_table(N, [1.2e4, 2.9e4])
    grp = rng.integers(0, 2, M).astype(np.int32)
    h = firm.ctf_weights(N, M, grp, table)
    Ker = firm.kernel_direct(N, R, h)
    offs = np.concatenate([rng.integers(-N + 1, N, size=(10, 3)),
                           [[N - 1, -(N - 1), 1], [-(N - 1), N - 1, -(N - 1)], [0, 0, 0], [3, -2, 0]]])
    ref = np.array([firm.kernel_value(Ker, N, o) for o in offs])
    scale = np.sum(h * h)
    assert np.max(np.abs(firm.kernel_at(offs, N, R, h) - ref)) <= 1e-11 * scale
    assert np.max(np.abs(direct.kernel_at(offs, N, R, grp, table) - ref)) <= 1e-9 * scale


@pytest.mark.parametrize("N,M", [(8, 4), (16, 3)])
def test_back_project_at_matches_full_back_projection(N, M):
    """The sampled direct sums of eq. backprojection (numpy and C, with CTF and re-centring of
    shifted images) equal the full-array A*, which is pinned by the adjoint identity with A and
    the projection-slice theorem.  Non-Hermitian data, so a sign slip in the phase shows."""
    rng = _rng(40 + N)
    R = synth.haar_rotations(M, rng)
    table = synth.ctf_table(N, [1.5e4, 2.4e4])
    grp = rng.integers(0, 2, M).astype(np.int32)
    h = firm.ctf_weights(N, M, grp, table)
    P = firm.slice_point_count(N)
    b = (rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))).astype(np.complex64)
    sh = rng.uniform(-2, 2, size=(M, 2))
    g = firm.recentre(b.astype(np.complex128), N, sh)
    full = firm.back_project(g, N, R, h)
    vox = np.concatenate([rng.integers(-N // 2, N // 2, size=(10, 3)),
                          [[-N // 2, -N // 2, -N // 2], [N // 2 - 1, N // 2 - 1, N // 2 - 1], [0, 0, 0]]])
    ref = np.array([full[v[0] + N // 2, v[1] + N // 2, v[2] + N // 2] for v in vox])
    scale = np.sum(np.abs(b))
    assert np.max(np.abs(firm.back_project_at(vox, g, N, R, h) - ref)) <= 1e-11 * scale
    assert np.max(np.abs(direct.backproject_at(vox, b, N, R, grp, table, sh) - ref)) <= 1e-9 * scale
    # the shift enters with the re-centring sign: without it the values differ at O(1)
    wrong = firm.back_project_at(vox, firm.recentre(b.astype(np.complex128), N, -sh), N, R, h)
    assert np.max(np.abs(wrong - ref)) > 1e-2 * np.max(np.abs(ref))


# ------------------------------------------------ FSC shells (section 4) --

# Plane waves cos(2 pi <j, n> / N + phase) at N = 16, each placing its power at +-j.  The shell
# of each j is read off by hand from |j| and the shell bounds 0.5 + (i-1) <= |j| < 0.5 + i of
# section 4 (the paper's eps = 1e-4 moves no lattice point: |j|^2 is an integer).  None: |j|
# outside shells 1 .. N/2 - 1 (the mean, and |j| >= 7.5).
_FSC_WAVES = [
    # j          |j|     shell  amplitude  sign in V1
    ((1, 0, 0), 1, 1.0, +1), ((1, 1, 0), 1, 0.5, -1),
    ((1, 1, 1), 2, 1.0, +1), ((2, 0, 0), 2, 2.0, +1), ((2, 1, 1), 2, 1.5, -1),
    ((2, 2, 0), 3, 1.0, -1), ((3, 0, 0), 3, 1.0, -1), ((2, 2, 2), 3, 0.7, -1),
    ((3, 2, 1), 4, 1.0, +1), ((4, 1, 1), 4, 1.0, -1),
    ((4, 2, 2), 5, 2.0, +1), ((4, 3, 0), 5, 1.0, +1),
    ((6, 0, 0), 6, 1.0, -1), ((5, 3, 1), 6, 3.0, +1),
    ((7, 0, 0), 7, 1.0, +1), ((7, 2, 0), 7, 1.0, +1), ((6, 3, 2), 7, 2.0, -1),
    ((0, 0, 0), None, 5.0, -1), ((7, 3, 0), None, 4.0, -1), ((8, 0, 0), None, 4.0, -1),
]


def test_fsc_shell_membership():
    N = 16
    rng = _rng(18)
    n = np.indices((N, N, N)) - N // 2
    V1 = np.zeros((N, N, N))
    V2 = np.zeros((N, N, N))
    num = np.zeros(N // 2)
    den = np.zeros(N // 2)
    for j, shell, a, s in _FSC_WAVES:
        wave = a * np.cos(2 * np.pi * np.tensordot(np.array(j), n, axes=1) / N + rng.uniform(0, 2 * np.pi))
        V1 += s * wave
        V2 += wave
        if shell is not None:
            num[shell] += s * a * a
            den[shell] += a * a
    got = firm.fsc(V1, V2)
    assert got.shape == (N // 2 - 1,)
    assert np.allclose(got, num[1:] / den[1:], atol=1e-12)


# ------------------------------------------------ noise level (SNR reading) --

def test_noise_sigma_closed_form():
    """SNR = mean clean power per Fourier sample / noise power per sample."""
    rng = _rng(19)
    M, P = 7, 113
    c1, c2 = 3.0, 0.5
    mag = np.where(rng.uniform(size=(M, P)) < 0.5, c1, c2)
    b = mag * np.exp(1j * rng.uniform(0, 2 * np.pi, size=(M, P)))
    snr = 0.05
    expect = math.sqrt(np.mean(mag ** 2) / snr)
    assert abs(firm.noise_sigma(b, snr) - expect) <= 1e-12 * expect
    b1 = 2.0 * np.exp(1j * rng.uniform(0, 2 * np.pi, size=(M, P)))
    assert abs(firm.noise_sigma(b1, 4.0) - 1.0) <= 1e-12
    assert firm.noise_sigma(b, float("inf")) == 0.0


def test_noise_at_sigma_realises_the_snr():
    """Hermitian noise drawn at noise_sigma(b, snr) has clean/noise power ratio snr (to the
    sampling error of 4e5 draws)."""
    rng = _rng(20)
    N, M = 32, 500
    P = firm.slice_point_count(N)
    b = (rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))) * 0.3
    snr = 1.0 / 30.0
    nz = firm.hermitian_noise(N, M, rng.standard_normal((M, P, 2)), firm.noise_sigma(b, snr))
    ratio = np.mean(np.abs(b) ** 2) / np.mean(np.abs(nz) ** 2)
    assert abs(ratio / snr - 1.0) < 0.01


# ------------------------------------------------ Fourier-space regularizer (section 5) --

def _stencil_zero_boundary(x):
    """6 x(n) - sum of the six neighbours, with zero values outside the volume."""
    xp = np.pad(x, 1)
    c = xp[1:-1, 1:-1, 1:-1]
    nb = (xp[2:, 1:-1, 1:-1] + xp[:-2, 1:-1, 1:-1] + xp[1:-1, 2:, 1:-1] + xp[1:-1, :-2, 1:-1]
          + xp[1:-1, 1:-1, 2:] + xp[1:-1, 1:-1, :-2])
    return 6.0 * c - nb


def _stencil_periodic(x):
    return 6.0 * x - sum(np.roll(x, s, axis=a) for a in range(3) for s in (1, -1))


def test_regularizer_order1_is_the_dirichlet_laplacian_stencil():
    x = _rng(50).standard_normal((8, 8, 8))
    assert np.max(np.abs(firm.regularizer_apply(x, 1) - _stencil_zero_boundary(x))) <= 1e-12


def test_regularizer_order2_is_the_periodic_stencil_twice_on_the_padded_grid():
    N = 8
    x = _rng(51).standard_normal((N, N, N))
    xp = np.zeros((2 * N,) * 3)
    xp[:N, :N, :N] = x
    ref = _stencil_periodic(_stencil_periodic(xp))[:N, :N, :N]
    assert np.max(np.abs(firm.regularizer_apply(x, 2) - ref)) <= 1e-11


def test_regularizer_kernel_taps_and_toeplitz_form():
    N = 8
    r1 = firm.regularizer_kernel(N, 1)
    ref = np.zeros_like(r1)
    c = N - 1
    ref[c, c, c] = 6.0
    for a in range(3):
        for sgn in (1, -1):
            idx = [c, c, c]
            idx[a] += sgn
            ref[tuple(idx)] = -1.0
    assert np.max(np.abs(r1 - ref)) <= 1e-12
    r2 = firm.regularizer_kernel(N, 2)
    o = np.indices(r2.shape) - c
    assert np.max(np.abs(r2[np.abs(o).sum(0) > 2])) <= 1e-12 and abs(r2.sum()) <= 1e-10
    assert abs(r2[c, c, c] - 42.0) <= 1e-10          # 6^2 + 6 (each neighbour squared)
    x = _rng(52).standard_normal((N, N, N))
    for p, r in ((1, r1), (2, r2), (3, firm.regularizer_kernel(N, 3))):
        y = firm.toeplitz_apply_fft(r, x).real
        assert np.max(np.abs(y - firm.regularizer_apply(x, p))) <= 1e-10
        assert float(np.sum(x * y)) >= 0.0            # positive semidefinite


# ------------------------------------------------ random conical tilt and the missing cone --

def test_rct_views_and_missing_cone():
    """Every RCT viewing direction is at the tilt angle from e3, the rotations are proper, and no
    sample point of any slice falls inside the cone of half-angle 90 - tilt about e3."""
    rng = _rng(60)
    R = synth.rct_rotations(500, 60.0, rng)
    assert np.allclose(R[:, 2, 2], 0.5, atol=1e-12)
    assert np.allclose(np.einsum("mij,mkj->mik", R, R), np.eye(3), atol=1e-12)
    assert np.allclose(np.linalg.det(R), 1.0)
    xi = firm.sample_points(16, R).reshape(-1, 3)
    r = np.linalg.norm(xi, axis=1)
    nz = r > 0
    polar = np.degrees(np.arccos(np.abs(xi[nz, 2]) / r[nz]))
    assert polar.min() >= 30.0 - 1e-9
    assert polar.min() <= 30.0 + 0.5          # the cone's edge is reached


def test_fsc_cone_membership():
    """Plane waves placed inside and outside a 30-degree cone about the third axis: the modified
    FSC keeps each one in its own region (cone membership by hand from the angle to e3)."""
    N = 16
    rng = _rng(61)
    n = np.indices((N, N, N)) - N // 2
    # j, shell, inside the 30-degree cone?, sign in V1
    waves = [((0, 0, 3), 3, True, -1), ((3, 0, 0), 3, False, +1), ((1, 0, 3), 3, True, +1),
             ((2, 0, 2), 3, False, -1), ((1, 1, 5), 5, True, -1), ((4, 1, 2), 5, False, +1),
             ((0, 2, 6), 6, True, +1), ((6, 0, 1), 6, False, -1)]
    V1 = np.zeros((N, N, N))
    V2 = np.zeros((N, N, N))
    for j, _, _, sg in waves:
        w = np.cos(2 * np.pi * np.tensordot(np.array(j), n, axes=1) / N + rng.uniform(0, 2 * np.pi))
        V1 += sg * w
        V2 += w
    for inside in (True, False):
        got = firm.fsc_cone(V1, V2, 30.0, inside)
        for i in range(1, N // 2):
            sel = [sg for j, sh, ins, sg in waves if sh == i and ins == inside]
            if sel:   # (shells without a wave correlate round-off only)
                assert abs(got[i - 1] - np.mean(sel)) <= 1e-12, (inside, i)
    assert np.allclose(firm.fsc_cone(V1, V2, 0.0, False), firm.fsc(V1, V2), equal_nan=True)
