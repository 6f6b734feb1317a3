"""Thin ctypes binding of libfirm (include/firm.h).

Argument marshalling only: every step runs in the HIP library.  Device buffers
are torch tensors on the ROCm device; the plan's stream is torch's current
stream unless one is given.  Importing this module loads libfirm.so and raises
if it has not been built (python -m paper_1307_5824_amd.build).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfirm.so")

FIRM_OK = 0
FIRM_ERR_ARG = 1
FIRM_ERR_ALLOC = 2
FIRM_ERR_HIP = 3
FIRM_ERR_STATE = 4
FIRM_ERR_BREAKDOWN = 5
FIRM_ERR_NOT_CONVERGED = 6
STATUS_NAMES = {0: "FIRM_OK", 1: "FIRM_ERR_ARG", 2: "FIRM_ERR_ALLOC", 3: "FIRM_ERR_HIP",
                4: "FIRM_ERR_STATE", 5: "FIRM_ERR_BREAKDOWN", 6: "FIRM_ERR_NOT_CONVERGED"}


class FirmOptions(ctypes.Structure):
    _fields_ = [("kb_width", ctypes.c_int), ("refine_every", ctypes.c_int), ("check_every", ctypes.c_int),
                ("precision", ctypes.c_int), ("lambda_relative", ctypes.c_int), ("khat_bf16", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("stream", ctypes.c_void_p), ("stagnation_iters", ctypes.c_int)]


class FirmCgReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("refinements", ctypes.c_int), ("fell_back", ctypes.c_int),
                ("status", ctypes.c_int), ("rel_res", ctypes.c_double), ("true_rel_res", ctypes.c_double),
                ("t_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FirmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1307_5824_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
    sig = {
        "firm_slice_points": (i64, [i]),
        "firm_plan_create": (i, [ctypes.POINTER(vp), i, i, vp, vp, vp, i, vp, ctypes.POINTER(FirmOptions)]),
        "firm_plan_destroy": (None, [vp]),
        "firm_plan_set_stream": (i, [vp, vp]),
        "firm_kernel_precompute": (i, [vp]),
        "firm_kernel_get": (i, [vp, vp]),
        "firm_kernel_set": (i, [vp, vp]),
        "firm_set_regularizer": (i, [vp, i, d]),
        "firm_synth_volume": (i, [vp, i, vp, vp, vp, vp]),
        "firm_fsc": (i, [vp, vp, vp, d, vp]),
        "firm_kernel_spectrum": (i, [vp, vp]),
        "firm_backproject": (i, [vp, vp, vp]),
        "firm_forward_project": (i, [vp, vp, vp]),
        "firm_images_to_slices": (i, [vp, vp, vp]),
        "firm_apply_AtA": (i, [vp, vp, vp, d]),
        "firm_apply_AtA_f64": (i, [vp, vp, vp, d]),
        "firm_apply_AtA_timed": (i, [vp, vp, vp, d, i, vp]),
        "firm_cg_solve": (i, [vp, vp, vp, d, d, i, vp, ctypes.POINTER(FirmCgReport)]),
        "firm_cg_solve_f64": (i, [vp, vp, vp, d, d, i, vp, ctypes.POINTER(FirmCgReport)]),
        "firm_precond_apply": (i, [vp, vp, vp, vp]),
        "firm_synth_slices": (i, [vp, i, vp, vp, vp, d, ctypes.c_uint64, vp]),
        "firm_synth_images": (i, [vp, i, vp, vp, vp, d, ctypes.c_uint64, vp]),
        "firm_last_error": (ctypes.c_char_p, [vp]),
        "firm_philox4x32_10": (None, [vp, vp, vp]),
        "firm_pcnet_num_params": (i64, []),
        "firm_pcnet_create": (i, [ctypes.POINTER(vp), i, vp]),
        "firm_pcnet_destroy": (None, [vp]),
        "firm_pcnet_set_params": (i, [vp, vp]),
        "firm_pcnet_get_params": (i, [vp, vp]),
        "firm_pcnet_forward": (i, [vp, vp, i, vp, i]),
        "firm_pcnet_loss_grad": (i, [vp, vp, i, i, i, i, vp, vp, vp, vp, vp, ctypes.POINTER(d), vp]),
        "firm_pcnet_train_step": (i, [vp, vp, i, i, i, i, vp, vp, vp, vp, vp, d, d, ctypes.POINTER(d)]),
        "firm_pcg_unrolled": (i, [vp, vp, vp, i, i, d, ctypes.POINTER(d), vp]),
        "firm_chan_spectrum": (i, [vp, d, vp]),
        "firm_pcnet_last_error": (ctypes.c_char_p, [vp]),
        "firm_kernel_features": (i, [vp, d, i, vp]),
        "firm_precond_from_output": (i, [vp, vp, i, vp, vp]),
        "firm_precond_from_output_noalloc": (i, [vp, vp, i, vp, vp]),
        "firm_probe_stats": (i, [vp, vp, i, d, vp, vp, ctypes.POINTER(d)]),
        "firm_synth_normals": (i, [vp, ctypes.c_uint64, ctypes.c_uint64, i64, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def last_error(plan=None):
    s = lib.firm_last_error(plan)
    return s.decode() if s else ""


def _check(status, plan=None):
    if status != FIRM_OK:
        raise FirmError(status, last_error(plan))
    return status


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _host(a, dtype):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    return arr, arr.ctypes.data_as(ctypes.c_void_p)


def firm_slice_points(N):
    return int(lib.firm_slice_points(N))


def firm_philox4x32_10(ctr, key):
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib.firm_philox4x32_10(c.ctypes.data_as(ctypes.c_void_p), k.ctypes.data_as(ctypes.c_void_p),
                           out.ctypes.data_as(ctypes.c_void_p))
    return out


def _current_stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def firm_plan_create(N, rotations, shifts=None, ctf_group=None, ctf_table=None, kb_width=0,
                     refine_every=0, check_every=0, stream=None, precision=0, lambda_relative=0, inner_tol=0.0,
                     khat_bf16=0, stagnation_iters=0):
    """Returns a raw plan handle (c_void_p); see Plan for the managed form."""
    rot, rotp = _host(np.asarray(rotations, dtype=np.float64).reshape(-1, 9), np.float64)
    M = rot.shape[0]
    sh, shp = _host(None if shifts is None else np.asarray(shifts).reshape(M, 2), np.float64)
    grp, grpp = _host(ctf_group, np.int32)
    tab, tabp = _host(ctf_table, np.float32)
    G = 0 if tab is None else (tab.shape[0] if tab.ndim == 2 else 1)
    opt = FirmOptions(kb_width, refine_every, check_every, precision, lambda_relative, int(khat_bf16), inner_tol,
                      stream, int(stagnation_iters))
    h = ctypes.c_void_p()
    _check(lib.firm_plan_create(ctypes.byref(h), int(N), int(M), rotp, shp, grpp, int(G), tabp, ctypes.byref(opt)))
    return h


class Plan:
    """Owns a firm_plan; device tensors are torch tensors on the current ROCm device."""

    def __init__(self, N, rotations, shifts=None, ctf_group=None, ctf_table=None, kb_width=0,
                 refine_every=0, check_every=0, stream=None, precision=0, lambda_relative=0, inner_tol=0.0,
                 khat_bf16=0, stagnation_iters=0):
        import torch
        self.N = int(N)
        self.M = int(np.asarray(rotations).reshape(-1, 9).shape[0])
        self.P = firm_slice_points(self.N)
        s = stream if stream is not None else _current_stream()
        self.h = firm_plan_create(N, rotations, shifts, ctf_group, ctf_table, kb_width, refine_every,
                                  check_every, s, precision, lambda_relative, inner_tol, khat_bf16, stagnation_iters)
        self._torch = torch

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib.firm_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vol(self, out=None, n=None):
        n = n or self.N
        if out is None:
            out = self._torch.empty((n, n, n), dtype=self._torch.float32, device="cuda")
        return out

    def _req(self, t, numel, dtype):
        if not t.is_cuda or not t.is_contiguous() or t.dtype != dtype or t.numel() != numel:
            raise ValueError(f"expected a contiguous {dtype} CUDA tensor of {numel} elements")
        return t

    def set_stream(self, stream):
        _check(lib.firm_plan_set_stream(self.h, stream), self.h)

    def kernel_precompute(self):
        _check(lib.firm_kernel_precompute(self.h), self.h)

    def kernel_get(self, out=None):
        out = self._vol(out, 2 * self.N)
        self._req(out, (2 * self.N) ** 3, self._torch.float32)
        _check(lib.firm_kernel_get(self.h, _ptr(out)), self.h)
        return out

    def kernel_set(self, ker):
        self._req(ker, (2 * self.N) ** 3, self._torch.float32)
        _check(lib.firm_kernel_set(self.h, _ptr(ker)), self.h)

    def set_regularizer(self, order, mu):
        """Fourier-space damping mu L_p added to A*A + lambda (order p in 0..3, mu like lambda)."""
        _check(lib.firm_set_regularizer(self.h, int(order), float(mu)), self.h)

    def kernel_spectrum(self, out=None):
        if out is None:
            out = self._torch.empty((2 * self.N, 2 * self.N, self.N + 1), dtype=self._torch.float32, device="cuda")
        self._req(out, 4 * self.N * self.N * (self.N + 1), self._torch.float32)
        _check(lib.firm_kernel_spectrum(self.h, _ptr(out)), self.h)
        return out

    def backproject(self, b, out=None):
        self._req(b, self.M * self.P, self._torch.complex64)
        out = self._vol(out)
        self._req(out, self.N ** 3, self._torch.float32)
        _check(lib.firm_backproject(self.h, _ptr(b), _ptr(out)), self.h)
        return out

    def forward_project(self, V, out=None):
        """Slices b (M x P complex64) of the volume V at the plan's views, CTFs and shifts."""
        self._req(V, self.N ** 3, self._torch.float32)
        if out is None:
            out = self._torch.empty((self.M, self.P), dtype=self._torch.complex64, device=V.device)
        self._req(out, self.M * self.P, self._torch.complex64)
        _check(lib.firm_forward_project(self.h, _ptr(V), _ptr(out)), self.h)
        return out

    def apply_AtA(self, x, lam, out=None):
        self._req(x, self.N ** 3, self._torch.float32)
        out = self._vol(out)
        self._req(out, self.N ** 3, self._torch.float32)
        _check(lib.firm_apply_AtA(self.h, _ptr(x), _ptr(out), float(lam)), self.h)
        return out

    def apply_AtA_timed(self, x, lam, reps, out=None):
        """Average ms of the five FFT passes of the product over reps runs."""
        self._req(x, self.N ** 3, self._torch.float32)
        out = self._vol(out)
        ms = (ctypes.c_float * 5)()
        _check(lib.firm_apply_AtA_timed(self.h, _ptr(x), _ptr(out), float(lam), int(reps), ms), self.h)
        return [float(v) for v in ms]

    def apply_AtA_f64(self, x, lam, out=None):
        self._req(x, self.N ** 3, self._torch.float64)
        if out is None:
            out = self._torch.empty((self.N,) * 3, dtype=self._torch.float64, device="cuda")
        self._req(out, self.N ** 3, self._torch.float64)
        _check(lib.firm_apply_AtA_f64(self.h, _ptr(x), _ptr(out), float(lam)), self.h)
        return out

    def cg_solve(self, atb, lam, tol, max_iter, x0=None, precond=None, raise_on_not_converged=False):
        """CG on (A*A + lam) x = atb.  A float32 atb runs firm_cg_solve (FP32 x); a float64 atb
        runs firm_cg_solve_f64 (FP64 x, precision 1 or 2)."""
        t = self._torch
        f64 = atb.dtype == t.float64
        self._req(atb, self.N ** 3, t.float64 if f64 else t.float32)
        x = t.zeros_like(atb) if x0 is None else x0.to(atb.dtype).clone()
        if precond is not None:
            self._req(precond, self.N ** 3, t.float32)
        rep = FirmCgReport()
        fn = lib.firm_cg_solve_f64 if f64 else lib.firm_cg_solve
        st = fn(self.h, _ptr(atb), _ptr(x), float(lam), float(tol), int(max_iter), _ptr(precond), ctypes.byref(rep))
        if st not in (FIRM_OK, FIRM_ERR_NOT_CONVERGED) or (st != FIRM_OK and raise_on_not_converged):
            raise FirmError(st, last_error(self.h))
        return x, rep.as_dict()

    def precond_apply(self, d, r, out=None):
        self._req(d, self.N ** 3, self._torch.float32)
        self._req(r, self.N ** 3, self._torch.float32)
        out = self._vol(out)
        _check(lib.firm_precond_apply(self.h, _ptr(d), _ptr(r), _ptr(out)), self.h)
        return out

    def images_to_slices(self, images, out=None):
        """Slices b (M x P complex64) from real images (M x N x N float32): Step 1."""
        self._req(images, self.M * self.N * self.N, self._torch.float32)
        if out is None:
            out = self._torch.empty((self.M, self.P), dtype=self._torch.complex64, device=images.device)
        self._req(out, self.M * self.P, self._torch.complex64)
        _check(lib.firm_images_to_slices(self.h, _ptr(images), _ptr(out)), self.h)
        return out

    def synth_images(self, centers, sigmas, amps, snr=float("inf"), seed=0, out=None):
        """Real-space projection images (M x N x N float32) of a blob volume at the plan's views
        and shifts, with white pixel noise at the given SNR."""
        c, cp = _host(np.asarray(centers).reshape(-1, 3), np.float64)
        s, sp = _host(np.ravel(sigmas), np.float64)
        a, ap = _host(np.ravel(amps), np.float64)
        if out is None:
            out = self._torch.empty((self.M, self.N, self.N), dtype=self._torch.float32, device="cuda")
        self._req(out, self.M * self.N * self.N, self._torch.float32)
        _check(lib.firm_synth_images(self.h, int(c.shape[0]), cp, sp, ap, float(snr), int(seed), _ptr(out)), self.h)
        return out

    def synth_volume(self, centers, sigmas, amps, out=None):
        """The sampled blob volume (N^3) whose slices synth_slices gives in closed form."""
        c, cp = _host(np.asarray(centers).reshape(-1, 3), np.float64)
        s, sp = _host(np.ravel(sigmas), np.float64)
        a, ap = _host(np.ravel(amps), np.float64)
        out = self._vol(out)
        _check(lib.firm_synth_volume(self.h, int(c.shape[0]), cp, sp, ap, _ptr(out)), self.h)
        return out

    def fsc(self, V1, V2, cone_deg=0.0):
        """Fourier shell correlation (section 4): (3, N/2 - 1) array, rows all shells' frequencies,
        outside and inside the cone of half-angle cone_deg about the third axis."""
        self._req(V1, self.N ** 3, self._torch.float32)
        self._req(V2, self.N ** 3, self._torch.float32)
        out = np.zeros(3 * (self.N // 2 - 1))
        _check(lib.firm_fsc(self.h, _ptr(V1), _ptr(V2), float(cone_deg), out.ctypes.data_as(ctypes.c_void_p)),
               self.h)
        return out.reshape(3, self.N // 2 - 1)

    def synth_slices(self, centers, sigmas, amps, snr=float("inf"), seed=0, out=None):
        c, cp = _host(np.asarray(centers).reshape(-1, 3), np.float64)
        s, sp = _host(np.ravel(sigmas), np.float64)
        a, ap = _host(np.ravel(amps), np.float64)
        if out is None:
            out = self._torch.empty((self.M, self.P), dtype=self._torch.complex64, device="cuda")
        self._req(out, self.M * self.P, self._torch.complex64)
        _check(lib.firm_synth_slices(self.h, int(c.shape[0]), cp, sp, ap, float(snr), int(seed), _ptr(out)), self.h)
        return out


# ---- learned preconditioner helpers (attached to Plan below)

def inference_res(N):
    """Network grid for a plan of size N: N / 4 within [32, 128].  The network sets a smooth floor
    under Chan's spectrum, so its grid hardly matters: at N = 256 on the large workload PCG takes 94
    iterations to 1e-5 at res 32, 64 and 128, and the network is fastest at res 64."""
    return int(min(128, max(32, N // 4)))


def _plan_kernel_features(self, lam_rel, res=32, out=None):
    if out is None:
        out = self._torch.empty((res, res, res), dtype=self._torch.float32, device="cuda")
    self._req(out, res ** 3, self._torch.float32)
    _check(lib.firm_kernel_features(self.h, float(lam_rel), int(res), _ptr(out)), self.h)
    return out


def _plan_precond_from_output(self, o, t, out=None):
    """d = 1 / (t + Ker(0) exp(U sym(o))) for a network output o (res^3) and the Fourier diagonal t."""
    res = int(o.shape[-1])
    self._req(o, res ** 3, self._torch.float32)
    self._req(t, self.N ** 3, self._torch.float32)
    out = self._vol(out)
    _check(lib.firm_precond_from_output(self.h, _ptr(o), res, _ptr(t), _ptr(out)), self.h)
    return out


def _plan_pcg_unrolled(self, d, probes, k, lam, with_grad=True, out=None):
    """Mean unrolled-PCG loss over the probes and (with_grad) its gradient in log d (N^3)."""
    t = self._torch
    P = probes.shape[0] if probes.dim() == 4 else 1
    self._req(probes, P * self.N ** 3, t.float32)
    self._req(d, self.N ** 3, t.float32)
    g = self._vol(out) if with_grad else None
    loss = ctypes.c_double()
    _check(lib.firm_pcg_unrolled(self.h, _ptr(d), _ptr(probes), int(P), int(k), float(lam), ctypes.byref(loss),
                                 _ptr(g)), self.h)
    return loss.value, g


def _plan_probe_stats(self, probes, lam):
    t = self._torch
    P = probes.shape[0]
    self._req(probes, P * self.N ** 3, t.float32)
    A = t.empty((self.N,) * 3, dtype=t.float32, device="cuda")
    B = t.empty_like(A)
    sc = ctypes.c_double()
    _check(lib.firm_probe_stats(self.h, _ptr(probes), int(P), float(lam), _ptr(A), _ptr(B), ctypes.byref(sc)), self.h)
    return A, B, sc.value


def _plan_chan_spectrum(self, lam, out=None):
    """Fourier diagonal of A*A + lam on the centred N^3 grid (T. Chan's circulant spectrum)."""
    out = self._vol(out)
    _check(lib.firm_chan_spectrum(self.h, float(lam), _ptr(out)), self.h)
    return out


def _plan_synth_normals(self, seed, offset, shape):
    t = self._torch
    out = t.empty(shape, dtype=t.float32, device="cuda")
    _check(lib.firm_synth_normals(self.h, int(seed), int(offset), int(out.numel()), _ptr(out)), self.h)
    return out


Plan.kernel_features = _plan_kernel_features
Plan.precond_from_output = _plan_precond_from_output
Plan.pcg_unrolled = _plan_pcg_unrolled
Plan.probe_stats = _plan_probe_stats
Plan.synth_normals = _plan_synth_normals
Plan.chan_spectrum = _plan_chan_spectrum


class PCNet:
    """The preconditioner network (device-resident FP32 masters, BF16 matrix-core copies)."""

    NPARAM = None

    def __init__(self, max_batch=8, stream=None):
        import torch
        self._torch = torch
        s = stream if stream is not None else _current_stream()
        h = ctypes.c_void_p()
        st = lib.firm_pcnet_create(ctypes.byref(h), int(max_batch), s)
        if st != FIRM_OK:
            raise FirmError(st, last_error())
        self.h = h
        self.max_batch = max_batch
        PCNet.NPARAM = int(lib.firm_pcnet_num_params())

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib.firm_pcnet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        if st != FIRM_OK:
            raise FirmError(st, (lib.firm_pcnet_last_error(self.h) or b"").decode())

    def set_params(self, params):
        arr = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
        assert arr.size == PCNet.NPARAM
        self._chk(lib.firm_pcnet_set_params(self.h, arr.ctypes.data_as(ctypes.c_void_p)))

    def get_params(self):
        arr = np.zeros(PCNet.NPARAM, dtype=np.float32)
        self._chk(lib.firm_pcnet_get_params(self.h, arr.ctypes.data_as(ctypes.c_void_p)))
        return arr

    def forward(self, feat):
        """Network output [B][res][res][res] for features [B][res][res][res] (or one [res]^3)."""
        t = self._torch
        B = feat.shape[0] if feat.dim() == 4 else 1
        res = int(feat.shape[-1])
        out = t.empty((B, res, res, res), dtype=t.float32, device="cuda")
        self._chk(lib.firm_pcnet_forward(self.h, _ptr(feat), res, _ptr(out), int(B)))
        return out

    OBJECTIVES = {"probe": 0, "kaporin": 1, "logd": 2}

    def loss_grad(self, feat, N, t, A=None, Bs=None, sumc=None, ker0=None, with_grad=True, objective="probe"):
        """Mean loss over the batch and (with_grad) the parameter gradients.  t: the Fourier
        diagonals [B][N^3]; objective "probe": A, Bs, sumc are probe statistics; "kaporin": no
        statistics; "logd": A is the gradient of the caller's loss in log d (the loss reads 0)."""
        B = feat.shape[0]
        sc = None if sumc is None else np.ascontiguousarray(np.asarray(sumc, dtype=np.float64))
        k0 = np.ascontiguousarray(np.asarray(ker0, dtype=np.float64))
        loss = ctypes.c_double()
        g = np.zeros(PCNet.NPARAM, dtype=np.float32) if with_grad else None
        self._chk(lib.firm_pcnet_loss_grad(self.h, _ptr(feat), int(feat.shape[-1]), int(B), int(N),
                                           self.OBJECTIVES[objective], _ptr(t), _ptr(A),
                                           _ptr(Bs), None if sc is None else sc.ctypes.data_as(ctypes.c_void_p),
                                           k0.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss),
                                           None if g is None else g.ctypes.data_as(ctypes.c_void_p)))
        return loss.value, g

    def train_step(self, feat, N, t, A=None, Bs=None, sumc=None, ker0=None, lr=1e-3, objective="probe",
                   lr_floor=None):
        """One Adam step; lr_floor (default lr) is the step of the output bias, the floor's level."""
        B = feat.shape[0]
        sc = None if sumc is None else np.ascontiguousarray(np.asarray(sumc, dtype=np.float64))
        k0 = np.ascontiguousarray(np.asarray(ker0, dtype=np.float64))
        loss = ctypes.c_double()
        self._chk(lib.firm_pcnet_train_step(self.h, _ptr(feat), int(feat.shape[-1]), int(B), int(N),
                                            self.OBJECTIVES[objective], _ptr(t), _ptr(A),
                                            _ptr(Bs), None if sc is None else sc.ctypes.data_as(ctypes.c_void_p),
                                            k0.ctypes.data_as(ctypes.c_void_p), float(lr),
                                            float(lr if lr_floor is None else lr_floor), ctypes.byref(loss)))
        return loss.value
