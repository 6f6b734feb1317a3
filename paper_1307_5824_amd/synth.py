"""Seeded synthetic inputs of the shape of the paper's cryo-EM workloads.

This module draws inputs only: rotations, shifts, defocus-group assignments,
CTF tables, Gaussian-blob parameters and raw normal variates.  It contains none
of the reconstruction arithmetic (no sample points, projections, kernels or
solvers), so the library and its FP64 checker can both take their inputs from
here without sharing any of the method.

Workload recipes (the paper's experiment, section 4, uses a 90^3 ribosome map,
10,000 random-conical-tilt projections, 3 defocus groups and SNR 1; that map
and those projections are not available, so sums of Gaussian blobs with
random orientations stand in for them):

  small    N=16,  5 blobs,   M=200,     Haar views, no shifts, no CTF, noiseless, lambda=1e-3
  mid      N=64,  40 blobs,  M=10,000,  Haar views, shifts U[-2,2], 10 groups, SNR 1/10, lambda=1e-2
  uneven   N=128, 100 blobs, M=50,000,  90% vMF(kappa=5) + 10% Haar, 20 groups, SNR 1/20, lambda=1e-2
  train    N=64,  per set kappa~U[0,20], 1..20 groups, M=10,000 (preconditioner training)
  large    N=256, 300 blobs, M=100,000, vMF(kappa=10), 50 groups, SNR 1/30, lambda=1e-2
  rct      N=256, 300 blobs, M=100,000, random conical tilt at 60 degrees (the paper's experiment
           geometry), 3 groups, SNR 1, lambda=1e-2
"""
import dataclasses

import numpy as np

BASE_SEED = 13075824


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    N: int
    blobs: int
    M: int
    kappa: float          # 0 = Haar-uniform views
    uniform_frac: float   # fraction of Haar views mixed into a vMF set
    shift_px: float       # shifts ~ U[-shift_px, shift_px]^2
    groups: int           # 0 = no CTF (h = 1)
    snr: float            # inf = noiseless
    lam: float
    index: int
    tilt_deg: float = 0.0  # > 0: random conical tilt series at this tilt, uniform azimuth


WORKLOADS = {
    "small": Workload("small", 16, 5, 200, 0.0, 0.0, 0.0, 0, float("inf"), 1e-3, 0),
    "mid": Workload("mid", 64, 40, 10_000, 0.0, 0.0, 2.0, 10, 0.1, 1e-2, 1),
    "uneven": Workload("uneven", 128, 100, 50_000, 5.0, 0.1, 2.0, 20, 0.05, 1e-2, 2),
    "train": Workload("train", 64, 40, 10_000, -1.0, 0.1, 2.0, -1, 0.1, 1e-2, 3),
    "large": Workload("large", 256, 300, 100_000, 10.0, 0.0, 2.0, 50, 1.0 / 30.0, 1e-2, 4),
    "rct": Workload("rct", 256, 300, 100_000, 0.0, 0.0, 2.0, 3, 1.0, 1e-2, 5, tilt_deg=60.0),
}


def streams(index, n=6):
    """Independent generators for (volume, rotations, shifts, ctf, noise, probes)."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(BASE_SEED + index).spawn(n)]


# --------------------------------------------------------------- rotations --

def quat_to_rot(q):
    """Rotation matrices from unit quaternions (w, x, y, z), shape (M, 3, 3)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def haar_rotations(M, rng):
    """Haar-uniform SO(3): normalised 4D Gaussian quaternions (Shoemake 1992)."""
    q = rng.standard_normal((M, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return quat_to_rot(q)


def vmf_directions(M, kappa, rng):
    """Unit vectors from the von Mises-Fisher distribution on S^2 about +e3 (Wood 1994)."""
    u = rng.random(M)
    if kappa <= 0:
        w = 2 * u - 1
    else:
        w = 1.0 + np.log(u + (1.0 - u) * np.exp(-2.0 * kappa)) / kappa
    w = np.clip(w, -1.0, 1.0)
    phi = rng.random(M) * 2 * np.pi
    s = np.sqrt(1 - w * w)
    return np.stack([s * np.cos(phi), s * np.sin(phi), w], axis=1)


def rotations_with_directions(d, rng):
    """Rotations whose third row (the viewing direction) is d, with a uniform in-plane angle."""
    M = d.shape[0]
    ref = np.where(np.abs(d[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    a = np.cross(d, ref)
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = np.cross(d, a)
    psi = rng.random(M) * 2 * np.pi
    r1 = np.cos(psi)[:, None] * a + np.sin(psi)[:, None] * b
    r2 = np.cross(d, r1)
    return np.stack([r1, r2, d], axis=1)


def rct_rotations(M, tilt_deg, rng):
    """A random conical tilt series (section 4): viewing directions at the tilt angle from +e3 with
    azimuths uniform in [0, 2 pi), uniform in-plane angles.  The slices then miss the cone of
    half-angle 90 - tilt degrees about e3 in Fourier space."""
    t = np.deg2rad(tilt_deg)
    phi = rng.random(M) * 2 * np.pi
    d = np.stack([np.sin(t) * np.cos(phi), np.sin(t) * np.sin(phi), np.full(M, np.cos(t))], axis=1)
    return rotations_with_directions(d, rng)


def mixed_rotations(M, kappa, uniform_frac, rng):
    """A fraction of Haar views, the rest vMF(kappa) about one pole; kappa 0 means all Haar."""
    if kappa == 0:
        return haar_rotations(M, rng)
    n_u = int(round(uniform_frac * M))
    R = np.empty((M, 3, 3))
    R[: M - n_u] = rotations_with_directions(vmf_directions(M - n_u, kappa, rng), rng)
    if n_u:
        R[M - n_u:] = haar_rotations(n_u, rng)
    return R[rng.permutation(M)]


# ------------------------------------------------------------------ CTF --

def electron_wavelength(kv):
    """Relativistic electron wavelength in Angstrom for an accelerating voltage in kV."""
    V = kv * 1e3
    return 12.2643247 / np.sqrt(V * (1 + 0.978466e-6 * V))


def ctf_table(N, defoci_A, pixel_A=3.0, kv=300.0, cs_mm=2.0, amp=0.07):
    """CTF lookup table H[g, q], q = k1^2 + k2^2 in [0, N^2/4]: the radial sinusoid of the
    paper's CTF model (section 3.1) with the wavelength on the defocus term and no envelope,
    h(r) = sin(-pi (df lambda r^2 - Cs lambda^3 r^4 / 2) - A), r = sqrt(q) / (N pixel) 1/A."""
    lam = electron_wavelength(kv)
    cs = cs_mm * 1e7
    q = np.arange(N * N // 4 + 1, dtype=np.float64)
    r2 = q / (N * pixel_A) ** 2
    df = np.asarray(defoci_A, dtype=np.float64)[:, None]
    chi = np.pi * (df * lam * r2 - 0.5 * cs * lam ** 3 * r2 * r2)
    return np.sin(-chi - amp).astype(np.float32)


def defoci(G, rng):
    """One defocus per group, U[1, 3] micrometre, in Angstrom."""
    return rng.uniform(1.0e4, 3.0e4, size=G)


# ----------------------------------------------------------------- volume --

def blob_params(N, B, rng):
    """Blob centres uniform in the ball of radius N/4 voxels (radius 0.5 of the box half-width),
    widths U[0.05, 0.15] N voxels and amplitudes U[0.5, 1]."""
    d = rng.standard_normal((B, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = (N / 4.0) * rng.random(B) ** (1.0 / 3.0)
    centers = d * rad[:, None]
    sigmas = rng.uniform(0.05, 0.15, size=B) * N
    amps = rng.uniform(0.5, 1.0, size=B)
    return centers, sigmas, amps


# ------------------------------------------------------------------ all --

@dataclasses.dataclass
class Inputs:
    workload: Workload
    rotations: np.ndarray      # (M, 3, 3) float64
    shifts: np.ndarray         # (M, 2) float64 or None
    ctf_group: np.ndarray      # (M,) int32 or None
    ctf_table: np.ndarray      # (G, N^2/4 + 1) float32 or None
    centers: np.ndarray
    sigmas: np.ndarray
    amps: np.ndarray
    noise_rng: np.random.Generator
    probe_rng: np.random.Generator


def make_inputs(workload, M=None, set_index=None):
    """All seeded inputs of a workload; M overrides the image count (smaller test sets).
    set_index selects one of the independent training / held-out sets of the 'train' recipe."""
    wl = WORKLOADS[workload] if isinstance(workload, str) else workload
    idx = wl.index if set_index is None else 1000 + wl.index * 100000 + set_index
    rv, rr, rs, rc, rn, rp = streams(idx)
    M = wl.M if M is None else M
    kappa, groups = wl.kappa, wl.groups
    if kappa < 0:                      # per-set draws of the training recipe
        kappa = float(rr.uniform(0.0, 20.0))
        groups = int(rc.integers(1, 21))
    R = rct_rotations(M, wl.tilt_deg, rr) if wl.tilt_deg > 0 else mixed_rotations(M, kappa, wl.uniform_frac, rr)
    shifts = rs.uniform(-wl.shift_px, wl.shift_px, size=(M, 2)) if wl.shift_px > 0 else None
    if groups > 0:
        table = ctf_table(wl.N, defoci(groups, rc))
        grp = rc.integers(0, groups, size=M).astype(np.int32)
    else:
        table, grp = None, None
    c, s, a = blob_params(wl.N, wl.blobs, rv)
    return Inputs(wl, R, shifts, grp, table, c, s, a, rn, rp)
