"""FP64 oracle for the FIRM operators (test infrastructure only; see package doc).

Conventions (all from section 2 and 3 of the paper):
  * Volume V is an N x N x N array; entry V[i1, i2, i3] is voxel n = i - N/2,
    -N/2 <= n_d < N/2 (section 3.1, volume sampling).
  * Slice frequencies omega_k = 2 pi (k1, k2) / N for lattice points k with
    ||k|| <= N/2 (section 3.1, eq. truncation).  The disk is enumerated in the
    canonical order: k1 ascending, and within a row k2 ascending.
  * Sample point xi_{k,m} = R_m^{-1} (omega_k1, omega_k2, 0)  (eq. forward-projector).
  * CTF weight h_m(||omega_k||) is read from a table indexed by the group of
    image m and by q = k1^2 + k2^2 (the CTF depends on the frequency magnitude
    only, section 3.1).

Readings (the paper does not fix these):
  * Shifts: image m is the projection translated by s_m pixels, so its slice
    carries the factor exp(-i <omega_k, s_m>); re-centring (section 3.1)
    multiplies b by exp(+i <omega_k, s_m>) before back-projection.
  * Circulant embedding (eq. embedding_circulant / embedding_index): read with
    0-based positions p in [0, 2N): offset p for p < N, p - 2N for p > N, and the
    wrap position p = N carries 0.  The cropped product never uses that slot.
  * Regularizer: (A*A + lambda I) x = A*b with lambda taken literally.
"""
import numpy as np


# ---------------------------------------------------------------- geometry --

def disk_points(N):
    """Lattice points k = (k1, k2) with ||k|| <= N/2 (eq. truncation), canonical order."""
    r = np.arange(-(N // 2), N // 2 + 1)
    k1, k2 = np.meshgrid(r, r, indexing="ij")
    inside = 4 * (k1 * k1 + k2 * k2) <= N * N
    return k1[inside].astype(np.int64), k2[inside].astype(np.int64)


def slice_point_count(N):
    """P(N): number of Fourier samples per image."""
    return disk_points(N)[0].size


def slice_frequencies(N):
    """omega_k = 2 pi k / N for the disk points, shape (P, 2)."""
    k1, k2 = disk_points(N)
    return 2.0 * np.pi * np.stack([k1, k2], axis=1).astype(np.float64) / N


def sample_points(N, rotations):
    """xi_{k,m} = R_m^{-1} (omega_k1, omega_k2, 0)^T, shape (M, P, 3) (eq. forward-projector)."""
    rotations = np.asarray(rotations, dtype=np.float64).reshape(-1, 3, 3)
    om = slice_frequencies(N)
    w3 = np.concatenate([om, np.zeros((om.shape[0], 1))], axis=1)          # (P, 3)
    rinv = np.linalg.inv(rotations)                                          # (M, 3, 3)
    return np.einsum("mij,pj->mpi", rinv, w3)


def ctf_weights(N, M, ctf_group=None, ctf_table=None):
    """h_m(||omega_k||) as an (M, P) array; no table means h = 1 (no CTF)."""
    P = slice_point_count(N)
    if ctf_table is None:
        return np.ones((M, P))
    k1, k2 = disk_points(N)
    q = k1 * k1 + k2 * k2
    table = np.asarray(ctf_table, dtype=np.float64)
    g = np.zeros(M, dtype=np.int64) if ctf_group is None else np.asarray(ctf_group, dtype=np.int64)
    return table[g][:, q]


def shift_phase(N, shifts):
    """exp(+i <omega_k, s_m>): the re-centring factor for translated images, shape (M, P)."""
    om = slice_frequencies(N)
    s = np.asarray(shifts, dtype=np.float64).reshape(-1, 2)
    return np.exp(1j * (s @ om.T))


def voxel_coords(N):
    """n = i - N/2 for i in [0, N)."""
    return np.arange(N, dtype=np.float64) - N // 2


# ------------------------------------------------------- A, A*, Ker direct --

def _chunks(total, size):
    for a in range(0, total, size):
        yield a, min(total, a + size)


def forward_project_at(V, xi, chunk=4096):
    """sum_n V_n exp(-i <n, xi_j>) at arbitrary points xi (J, 3): the sum of eq. forward-projector.

    The sum over n is the separable product of the three per-axis phase
    factors exp(-i n_d xi_d); it is contracted one axis at a time.
    """
    V = np.asarray(V)
    N = V.shape[0]
    pts = np.asarray(xi, dtype=np.float64).reshape(-1, 3)
    n = voxel_coords(N)
    out = np.empty(pts.shape[0], dtype=np.complex128)
    for a, b in _chunks(pts.shape[0], chunk):
        e1 = np.exp(-1j * np.outer(pts[a:b, 0], n))
        e2 = np.exp(-1j * np.outer(pts[a:b, 1], n))
        e3 = np.exp(-1j * np.outer(pts[a:b, 2], n))
        t = np.einsum("abc,jc->jab", V, e3)            # sum over n3
        t = np.einsum("jab,jb->ja", t, e2)             # sum over n2
        out[a:b] = np.einsum("ja,ja->j", t, e1)        # sum over n1
    return out


def forward_project(V, rotations, h=None, chunk=4096):
    """(A V)(k, m) = sum_n V_n exp(-i <n, xi_{k,m}>) h_m(||omega_k||)  (eq. forward-projector)."""
    N = np.asarray(V).shape[0]
    xi = sample_points(N, rotations)
    M, P, _ = xi.shape
    out = forward_project_at(V, xi.reshape(-1, 3), chunk)
    out = out.reshape(M, P)
    if h is not None:
        out = out * h
    return out


def back_project(g, N, rotations, h=None, chunk=4096):
    """(A* g)(n) = sum_m sum_k exp(+i <n, xi_{k,m}>) h_m g_{k,m}  (eq. backprojection). Complex N^3."""
    xi = sample_points(N, rotations)
    M, P, _ = xi.shape
    g = np.asarray(g, dtype=np.complex128).reshape(M, P)
    c = (g * h if h is not None else g).reshape(-1)
    pts = xi.reshape(-1, 3)
    n = voxel_coords(N)
    out = np.zeros((N, N, N), dtype=np.complex128)
    for a, b in _chunks(pts.shape[0], chunk):
        e1 = np.exp(1j * np.outer(pts[a:b, 0], n))
        e2 = np.exp(1j * np.outer(pts[a:b, 1], n))
        e3 = np.exp(1j * np.outer(pts[a:b, 2], n))
        t = (c[a:b, None] * e1)                        # (j, n1)
        t = np.einsum("ja,jb->jab", t, e2)             # (j, n1, n2)
        out += np.einsum("jab,jc->abc", t, e3)
    return out


def recentre(b, N, shifts):
    """Multiply slices by exp(+i <omega_k, s_m>) (images re-shifted to their centres, section 3.1)."""
    if shifts is None:
        return np.asarray(b, dtype=np.complex128)
    return np.asarray(b, dtype=np.complex128) * shift_phase(N, shifts)


def kernel_direct(N, rotations, h=None, chunk=2048):
    """Ker(n) = sum_m sum_k exp(+i <n, xi_{k,m}>) h_m^2 for -N < n < N  (eq. kernel).

    Returned as a complex (2N-1)^3 array indexed by n + N - 1.
    """
    xi = sample_points(N, rotations)
    M, P, _ = xi.shape
    w = (h * h if h is not None else np.ones((M, P))).reshape(-1)
    pts = xi.reshape(-1, 3)
    n = np.arange(-N + 1, N, dtype=np.float64)
    L = n.size
    out = np.zeros((L, L, L), dtype=np.complex128)
    for a, b in _chunks(pts.shape[0], chunk):
        e1 = np.exp(1j * np.outer(pts[a:b, 0], n)) * w[a:b, None]
        e2 = np.exp(1j * np.outer(pts[a:b, 1], n))
        e3 = np.exp(1j * np.outer(pts[a:b, 2], n))
        t = np.einsum("ja,jb->jab", e1, e2).reshape(b - a, L * L)
        out += (t.T @ e3).reshape(L, L, L)
    return out


def kernel_at(offsets, N, rotations, h=None):
    """Ker at a list of integer offsets (K, 3), each by the direct sum of eq. kernel."""
    xi = sample_points(N, rotations).reshape(-1, 3)
    M = np.asarray(rotations).reshape(-1, 9).shape[0]
    P = slice_point_count(N)
    w = (h * h if h is not None else np.ones((M, P))).reshape(-1)
    offs = np.asarray(offsets, dtype=np.float64).reshape(-1, 3)
    return np.array([np.sum(w * np.exp(1j * (xi @ o))) for o in offs])


def back_project_at(voxels, g, N, rotations, h=None):
    """(A* g)(n) at a list of voxel offsets n (K, 3) by the direct sum of eq. backprojection."""
    xi = sample_points(N, rotations).reshape(-1, 3)
    M = np.asarray(rotations).reshape(-1, 9).shape[0]
    P = slice_point_count(N)
    c = np.asarray(g, dtype=np.complex128).reshape(M, P)
    if h is not None:
        c = c * h
    c = c.reshape(-1)
    vox = np.asarray(voxels, dtype=np.float64).reshape(-1, 3)
    return np.array([np.sum(c * np.exp(1j * (xi @ v))) for v in vox])


# ------------------------------------------------------------ Toeplitz apply --

def kernel_value(Ker, N, d):
    """Ker at offset d (three ints in (-N, N)) from a (2N-1)^3 array."""
    return Ker[d[0] + N - 1, d[1] + N - 1, d[2] + N - 1]


def toeplitz_apply_brute(Ker, x):
    """(Ker * x)(n) = sum_l x_l Ker(n - l), n, l in the N^3 grid (eq. toeplitz / toep2)."""
    x = np.asarray(x)
    N = x.shape[0]
    out = np.zeros((N, N, N), dtype=np.result_type(Ker, x, np.float64))
    idx = np.arange(N)
    for l1 in range(N):
        for l2 in range(N):
            for l3 in range(N):
                v = x[l1, l2, l3]
                if v == 0:
                    continue
                out += v * Ker[np.ix_(idx - l1 + N - 1, idx - l2 + N - 1, idx - l3 + N - 1)]
    return out


def circulant_first_column(Ker, N):
    """First column of the 2N-per-axis circulant embedding C^A (eq. embedding_circulant).

    Position p in [0, 2N) holds offset o(p) = p (p < N) or p - 2N (p > N); the
    wrap position p = N holds 0 (reading of eq. embedding_index, see module doc).
    """
    c = np.zeros((2 * N,) * 3, dtype=Ker.dtype)
    p = np.arange(2 * N)
    valid = p != N
    off = np.where(p < N, p, p - 2 * N)
    pv = p[valid]
    ov = off[valid] + N - 1
    c[np.ix_(pv, pv, pv)] = Ker[np.ix_(ov, ov, ov)]
    return c


def toeplitz_apply_fft(Ker, x):
    """Ker * x through the 2N circulant embedding and 3D FFTs (eq. circ1 in three dimensions).

    The circulant C = F* Lambda F is diagonalised by the DFT; its eigenvalues are
    the DFT of the first column.  x is zero-padded to 2N per axis and the first
    N entries per axis of the product are kept.
    """
    x = np.asarray(x)
    N = x.shape[0]
    lam = np.fft.fftn(circulant_first_column(Ker, N))
    xp = np.zeros((2 * N,) * 3, dtype=np.complex128)
    xp[:N, :N, :N] = x
    y = np.fft.ifftn(lam * np.fft.fftn(xp))[:N, :N, :N]
    return y


def toeplitz_operator(Ker, workers=None):
    """x -> (Ker * x) for a real, even kernel Ker ((2N-1)^3, offsets -N+1..N-1) and real x: the
    product of toeplitz_apply_fft (the 2N circulant embedding, eq. circ1 in three dimensions), with
    the embedding's spectrum computed once and real-to-complex FFTs (scipy.fft on `workers` threads)
    so that N = 256 products take seconds.  The spectrum of a real even column is real."""
    import scipy.fft as sfft
    Ker = np.asarray(Ker, dtype=np.float64)
    N = (Ker.shape[0] + 1) // 2
    lam = sfft.rfftn(circulant_first_column(Ker, N), workers=workers).real

    def apply(x):
        xp = np.zeros((2 * N,) * 3)
        xp[:N, :N, :N] = x
        y = sfft.irfftn(lam * sfft.rfftn(xp, workers=workers), s=xp.shape, workers=workers)
        return y[:N, :N, :N]
    return apply


# ------------------------------------------------------- Fourier-space regularizer --

def laplacian_symbol(L):
    """w(q) = sum_d 4 sin^2(pi q_d / L) on the L-periodic grid, q in FFT order: the DFT of the
    7-point negative Laplacian stencil (6 at the centre, -1 at the six neighbours)."""
    a = 4.0 * np.sin(np.pi * np.arange(L) / L) ** 2
    return a[:, None, None] + a[None, :, None] + a[None, None, :]


def regularizer_apply(x, order):
    """L_p x = crop(F_2N^{-1}(w^p . F_2N(pad x))): the damping of high frequencies that section 5
    names as a Fourier-space regularizer, read as powers of the discrete Laplacian's symbol on the
    product's zero-padded 2N grid (the same pad and crop as the circulant embedding)."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    xp = np.zeros((2 * N,) * 3)
    xp[:N, :N, :N] = x
    y = np.fft.ifftn(laplacian_symbol(2 * N) ** order * np.fft.fftn(xp))
    return y[:N, :N, :N].real


def regularizer_kernel(N, order):
    """The Toeplitz kernel of L_p on offsets -N < o < N ((2N-1)^3, indexed like kernel_direct): the
    inverse DFT of w^p on the 2N grid read at its circulant positions (o mod 2N)."""
    c = np.fft.ifftn(laplacian_symbol(2 * N) ** order).real
    o = np.arange(-N + 1, N) % (2 * N)
    return c[np.ix_(o, o, o)]


def toeplitz_dense(Ker, N):
    """The N^3 x N^3 matrix T[(n), (l)] = Ker(n - l) (eq. toep3)."""
    i = np.indices((N, N, N)).reshape(3, -1)
    d = i[:, :, None] - i[:, None, :] + (N - 1)
    return Ker[d[0], d[1], d[2]]


# ------------------------------------------------------------ solvers --

def cg(apply, b, iters=None, tol=None, x0=None, record=False):
    """Conjugate gradients for the SPD system apply(x) = b (section 3.3), FP64.

    Stops after `iters` steps, or when ||b - apply(x)|| / ||b|| <= tol measured on
    the recursively updated residual.  Returns x (and the list of iterates and
    residual norms if record).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply(x) if x0 is not None else b.copy()
    p = r.copy()
    rr = float(np.vdot(r, r).real)
    nb = float(np.sqrt(np.vdot(b, b).real))
    hist, res = [x.copy()], [np.sqrt(rr) / nb]
    k = 0
    while True:
        if iters is not None and k >= iters:
            break
        if tol is not None and np.sqrt(rr) / nb <= tol:
            break
        q = apply(p)
        alpha = rr / float(np.vdot(p, q).real)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(np.vdot(r, r).real)
        p = r + (rr_new / rr) * p
        rr = rr_new
        k += 1
        if record:
            hist.append(x.copy())
            res.append(np.sqrt(rr) / nb)
    if record:
        return x, hist, res
    return x


def pcg(apply, precond, b, iters=None, tol=None, record=False):
    """Preconditioned CG with an SPD preconditioner z = precond(r), x0 = 0, FP64."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    z = precond(r)
    p = z.copy()
    rz = float(np.vdot(r, z).real)
    nb = float(np.sqrt(np.vdot(b, b).real))
    hist, res = [x.copy()], [1.0]
    k = 0
    while True:
        rn = float(np.sqrt(np.vdot(r, r).real)) / nb
        if iters is not None and k >= iters:
            break
        if tol is not None and rn <= tol:
            break
        q = apply(p)
        alpha = rz / float(np.vdot(p, q).real)
        x = x + alpha * p
        r = r - alpha * q
        z = precond(r)
        rz_new = float(np.vdot(r, z).real)
        p = z + (rz_new / rz) * p
        rz = rz_new
        k += 1
        if record:
            hist.append(x.copy())
            res.append(float(np.sqrt(np.vdot(r, r).real)) / nb)
    if record:
        return x, hist, res
    return x


def fourier_diagonal_precond(d):
    """z = F_N^{-1}(d . F_N r) on the periodic N^3 grid (eq. circ1: a circulant is diagonal in
    the Fourier basis).  d is indexed by centred frequency q + N/2, -N/2 <= q < N/2."""
    d = np.asarray(d, dtype=np.float64)
    ds = np.fft.ifftshift(d)           # centred order -> FFT order

    def apply(r):
        return np.fft.ifftn(ds * np.fft.fftn(r)).real
    return apply


def krylov_iterate(apply, b, k):
    """The k-th CG iterate in exact arithmetic: the minimiser of the energy-norm error over
    the Krylov space K_k(T, b), x0 = 0.  Built from an orthonormal basis with full
    re-orthogonalisation and a k x k solve (a definition of CG independent of its recursion)."""
    b = np.asarray(b, dtype=np.float64)
    shape = b.shape
    b = b.reshape(-1)

    def op(v):
        return np.asarray(apply(v.reshape(shape))).reshape(-1)
    Q = np.zeros((b.size, k))
    v = b / np.linalg.norm(b)
    for j in range(k):
        for _ in range(2):
            v = v - Q[:, :j] @ (Q[:, :j].T @ v)
        v = v / np.linalg.norm(v)
        Q[:, j] = v
        v = op(v)
    TQ = np.stack([op(Q[:, j]) for j in range(k)], axis=1)
    H = Q.T @ TQ
    H = 0.5 * (H + H.T)
    y = np.linalg.solve(H, Q.T @ b)
    return (Q @ y).reshape(shape)


def chan_circulant_spectrum(Ker, N, lam=0.0):
    """T. Chan's optimal circulant approximation of the N^3 Toeplitz operator (used by the
    analytic Fourier-diagonal preconditioner): first column
    c(j) = sum over the two offsets o in {j, j - N} of prod_d (1 - |o_d| / N) Ker(o), then
    its DFT; returned in centred frequency order, plus lam."""
    Kr = np.real(Ker)
    c = np.zeros((N, N, N))
    for a in range(N):
        for b_ in range(N):
            for cc in range(N):
                s = 0.0
                for o1 in (a, a - N):
                    if o1 == -N:
                        continue
                    for o2 in (b_, b_ - N):
                        if o2 == -N:
                            continue
                        for o3 in (cc, cc - N):
                            if o3 == -N:
                                continue
                            wgt = (1 - abs(o1) / N) * (1 - abs(o2) / N) * (1 - abs(o3) / N)
                            s += wgt * Kr[o1 + N - 1, o2 + N - 1, o3 + N - 1]
                c[a, b_, cc] = s
    return np.fft.fftshift(np.fft.fftn(c).real) + lam


# ------------------------------------------------------------ evaluation --

def fsc(V1, V2, eps=1e-4):
    """Fourier shell correlation (section 4): shells 0.5 + (i-1) + eps <= ||j|| < 0.5 + i + eps,
    i = 1 .. N/2 - 1."""
    N = V1.shape[0]
    F1 = np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(V1)))
    F2 = np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(V2)))
    j = np.indices((N, N, N)) - N // 2
    rad = np.sqrt((j * j).sum(0))
    out = []
    for i in range(1, N // 2):
        s = (rad >= 0.5 + (i - 1) + eps) & (rad < 0.5 + i + eps)
        num = np.sum(F1[s] * np.conj(F2[s]))
        den = np.sqrt(np.sum(np.abs(F1[s]) ** 2) * np.sum(np.abs(F2[s]) ** 2))
        out.append((num / den).real)
    return np.array(out)


def fsc_cone(V1, V2, cone_deg, inside, eps=1e-4):
    """The modified FSC of section 4: the shell sums restricted to the frequencies inside (or
    outside) the cone of half-angle cone_deg about the third axis, the missing cone of a random
    conical tilt series.  NaN where a shell has no such frequency."""
    N = V1.shape[0]
    F1 = np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(V1)))
    F2 = np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(V2)))
    j = np.indices((N, N, N)) - N // 2
    rad = np.sqrt((j * j).sum(0))
    in_cone = np.abs(j[2]) > rad * np.cos(np.deg2rad(cone_deg))
    region = in_cone if inside else ~in_cone
    out = []
    for i in range(1, N // 2):
        s = (rad >= 0.5 + (i - 1) + eps) & (rad < 0.5 + i + eps) & region
        num = np.sum(F1[s] * np.conj(F2[s]))
        den = np.sqrt(np.sum(np.abs(F1[s]) ** 2) * np.sum(np.abs(F2[s]) ** 2))
        out.append((num / den).real if den > 0 else np.nan)
    return np.array(out)


# ------------------------------------------------------------ noise --

def hermitian_noise(N, M, z, sigma):
    """Complex white noise on the disk with the symmetry of a real image's DFT:
    n(-k) = conj(n(k)) and n(0) real.  z is an (M, P, 2) array of raw standard normals;
    each sample has E|n|^2 = sigma^2.  The disk order is symmetric: index P-1-j holds -k_j."""
    P = slice_point_count(N)
    z = np.asarray(z, dtype=np.float64).reshape(M, P, 2)
    n = (z[..., 0] + 1j * z[..., 1]) * (sigma / np.sqrt(2.0))
    half = P // 2
    n[:, P - half:] = np.conj(n[:, :half][:, ::-1])
    n[:, half] = z[:, half, 0] * sigma
    return n


def noise_sigma(b_clean, snr):
    """Noise standard deviation per Fourier sample for a given SNR: mean clean power / SNR
    over all images and disk samples (equal to the real-space variance ratio by Parseval)."""
    if not np.isfinite(snr):
        return 0.0
    return float(np.sqrt(np.mean(np.abs(b_clean) ** 2) / snr))
