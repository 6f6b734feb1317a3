"""ctypes binding of direct.c: FP64 direct sums at sampled outputs (test infrastructure only).

The shared object is compiled with plain gcc (no fast-math) by `build()`; it is
built on first use if missing.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct.c")
_LIB = os.path.join(_HERE, "_direct.so")
_lib = None


def build():
    """Compile direct.c into oracle/_direct.so (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _LIB)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        p = ctypes.c_void_p
        i = ctypes.c_int
        lib.oracle_slice_points.restype = ctypes.c_int64
        lib.oracle_slice_points.argtypes = [i]
        lib.oracle_kernel_at.argtypes = [i, i, p, p, p, i, p, p, i]
        lib.oracle_backproject_at.argtypes = [i, i, p, p, p, p, p, i, p, p, i]
        lib.oracle_blob_slices.argtypes = [i, i, p, p, p, p, i, p, p, p, p, i]
        _lib = lib
    return _lib


def _threads(nthreads):
    return int(nthreads or os.cpu_count() or 1)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _prep(rotations, ctf_group, ctf_table):
    rot = np.ascontiguousarray(np.asarray(rotations, dtype=np.float64).reshape(-1, 9))
    grp = None if ctf_group is None else np.ascontiguousarray(np.asarray(ctf_group, dtype=np.int32))
    tab = None if ctf_table is None else np.ascontiguousarray(np.asarray(ctf_table, dtype=np.float32))
    return rot, grp, tab


def slice_points(N):
    return int(_load().oracle_slice_points(N))


def kernel_at(offsets, N, rotations, ctf_group=None, ctf_table=None, nthreads=None):
    """Ker(n) (complex) at integer offsets (K, 3) by the direct sum of eq. kernel."""
    rot, grp, tab = _prep(rotations, ctf_group, ctf_table)
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1, 3))
    out = np.zeros((offs.shape[0], 2))
    _load().oracle_kernel_at(N, rot.shape[0], _ptr(rot), _ptr(grp), _ptr(tab), offs.shape[0],
                             _ptr(offs), _ptr(out), _threads(nthreads))
    return out[:, 0] + 1j * out[:, 1]


def backproject_at(voxels, b, N, rotations, ctf_group=None, ctf_table=None, shifts=None, nthreads=None):
    """(A* recentre(b))(n) (complex) at voxel offsets n (K, 3); b is complex64 M x P."""
    rot, grp, tab = _prep(rotations, ctf_group, ctf_table)
    sh = None if shifts is None else np.ascontiguousarray(np.asarray(shifts, dtype=np.float64).reshape(-1, 2))
    bb = np.ascontiguousarray(np.asarray(b, dtype=np.complex64))
    vox = np.ascontiguousarray(np.asarray(voxels, dtype=np.int32).reshape(-1, 3))
    out = np.zeros((vox.shape[0], 2))
    _load().oracle_backproject_at(N, rot.shape[0], _ptr(rot), _ptr(grp), _ptr(tab), _ptr(sh), _ptr(bb),
                                  vox.shape[0], _ptr(vox), _ptr(out), _threads(nthreads))
    return out[:, 0] + 1j * out[:, 1]


def blob_slices(N, rotations, centers, sigmas, amps, ctf_group=None, ctf_table=None, shifts=None,
                nthreads=None):
    """Clean slices (M, P) complex128 of translated, CTF-filtered blob projections (closed form)."""
    rot, grp, tab = _prep(rotations, ctf_group, ctf_table)
    sh = None if shifts is None else np.ascontiguousarray(np.asarray(shifts, dtype=np.float64).reshape(-1, 2))
    c = np.ascontiguousarray(np.asarray(centers, dtype=np.float64).reshape(-1, 3))
    s = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64).reshape(-1))
    a = np.ascontiguousarray(np.asarray(amps, dtype=np.float64).reshape(-1))
    M = rot.shape[0]
    P = slice_points(N)
    out = np.zeros((M, P, 2))
    _load().oracle_blob_slices(N, M, _ptr(rot), _ptr(grp), _ptr(tab), _ptr(sh), c.shape[0], _ptr(c),
                               _ptr(s), _ptr(a), _ptr(out), _threads(nthreads))
    return out[..., 0] + 1j * out[..., 1]
