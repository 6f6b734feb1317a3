"""End-to-end runs of the mid (N = 64, 10^4 Haar views, 10 CTF groups) and uneven (N = 128,
5 * 10^4 views, 90% vMF kappa = 5 about one pole + 10% Haar, 20 CTF groups) workloads: kernel
precompute, back-projection and the solvers to 1e-5, each checked against the FP64 oracle.

* Ker at sampled offsets (the origin and the crop edges among them) against the direct sums of
  eq. kernel over every sample point with its CTF (oracle/direct.c).
* A*b at sampled voxels against the direct sums of eq. backprojection with re-centring, for
  seeded complex slices (all views at mid; 60 views of the uneven set, the rest zero, so the
  oracle's sum over those views is exact while the GPU runs the full launch).
* Plain CG, T. Chan PCG and the learned PCG (precision 1, lam = 1e-2 Ker(0), tol 1e-5): the
  FP32 solution's relative residual under the oracle's FP64 product with the plan's kernel (the
  operator the library solves, its values pinned by the sampled direct sums) is within tol.
* uneven, 16-bit kernel spectrum (both forms): the product within 1e-3 of the oracle's FP64
  product, and the FP64-refined solve to 1e-5 under the oracle.
* mid with lambda read literally (1e-2 absolute instead of relative to Ker(0)): plain CG stops at
  its 3000-iteration limit above 1e-5 (the reading the workloads do not take).
Tolerances as at full size: sampled values to 1e-5 relative L2 and 1e-5 Ker(0) each.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import rel  # noqa: E402
from oracle import direct as odirect  # noqa: E402
from oracle import firm as ofirm  # noqa: E402
from paper_1307_5824_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-5
WORKERS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def firm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1307_5824_amd import firm as f
    return f


def _offsets(N):
    return np.array([[0, 0, 0], [1, 0, 0], [0, 0, -1], [3, -2, 5], [-N // 4, N // 8, 7], [N // 2, -N // 3, N // 5],
                     [-(N - 1), 0, N - 1], [N - 1, -(N - 1), N // 2], [2, N - 2, -(N - 3)]])


def _at(vol, idx):
    t = torch.as_tensor(np.asarray(idx, dtype=np.int64)).cuda()
    out = vol[t[:, 0], t[:, 1], t[:, 2]]
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def _check_kernel(plan, inp, N):
    offs = _offsets(N)
    ref = odirect.kernel_at(offs, N, inp.rotations, inp.ctf_group, inp.ctf_table, nthreads=WORKERS).real
    got = _at(plan.kernel_get(), offs + N)
    err = np.abs(got - ref)
    print(f"  Ker: rel L2 {rel(got, ref):.2e}, max |err| / Ker(0) {err.max() / ref[0]:.2e}", flush=True)
    assert rel(got, ref) < TOL and err.max() <= TOL * ref[0]


def _check_backprojection(plan, inp, N, nviews, seed):
    M, P = plan.M, plan.P
    rng = np.random.default_rng(seed)
    views = np.arange(M) if nviews >= M else np.sort(rng.choice(M, nviews, replace=False))
    bv = (rng.standard_normal((len(views), P)) + 1j * rng.standard_normal((len(views), P))).astype(np.complex64)
    if nviews >= M:
        b = torch.as_tensor(bv).cuda()
    else:
        b = torch.zeros((M, P), dtype=torch.complex64, device="cuda")
        b[torch.as_tensor(views).cuda()] = torch.as_tensor(bv).cuda()
    atb = plan.backproject(b)
    del b
    vox = np.concatenate([rng.integers(0, N, (10, 3)), [[0, 0, 0], [N - 1, N - 1, N - 1], [N // 2] * 3]])
    got = _at(atb, vox)
    ref = odirect.backproject_at(vox - N // 2, bv, N, inp.rotations[views], inp.ctf_group[views], inp.ctf_table,
                                 inp.shifts[views], nthreads=WORKERS).real
    print(f"  A*b ({len(views)} views): rel L2 {rel(got, ref):.2e}", flush=True)
    assert rel(got, ref) < TOL


def _oracle_operator(plan, N, lam_rel):
    ker = plan.kernel_get()
    ker0 = float(ker[N, N, N])
    Kf = ker[1:, 1:, 1:].cpu().numpy().astype(np.float64)
    T = ofirm.toeplitz_operator(Kf, workers=WORKERS)
    lam = lam_rel * ker0

    def apply(x):
        return T(x) + lam * x
    return apply


def _check_solves(firm, plan, inp, N, apply, seed):
    from paper_1307_5824_amd import train_precond
    lam_rel = inp.workload.lam
    g = torch.Generator(device="cuda").manual_seed(seed)
    b = torch.randn((N, N, N), device="cuda", generator=g)
    bh = b.cpu().numpy().astype(np.float64)
    net = firm.PCNet(max_batch=1)
    net.set_params(train_precond.load_weights())
    t = plan.chan_spectrum(lam_rel)
    d = plan.precond_from_output(net.forward(plan.kernel_features(lam_rel, res=firm.inference_res(N))[None])[0], t)
    iters = {}
    for name, pc in (("cg", None), ("chan", torch.reciprocal(t)), ("learned", d)):
        x, rep = plan.cg_solve(b, lam_rel, TOL, 3000, precond=pc)
        xh = x.cpu().numpy().astype(np.float64)
        rr = float(np.linalg.norm(bh - apply(xh)) / np.linalg.norm(bh))
        print(f"  {name}: {rep['iters']} iterations, oracle rel res {rr:.3e} (library {rep['true_rel_res']:.3e})",
              flush=True)
        assert rep["status"] == 0 and rr <= TOL * 1.01
        iters[name] = rep["iters"]
    assert iters["learned"] < iters["cg"]
    return b, bh


def test_mid_workload_end_to_end(firm):
    inp = synth.make_inputs("mid")
    N = inp.workload.N
    print(f"mid: N={N} M={inp.rotations.shape[0]}", flush=True)
    plan = firm.Plan(N, inp.rotations, shifts=inp.shifts, ctf_group=inp.ctf_group, ctf_table=inp.ctf_table,
                     precision=1, lambda_relative=1)
    plan.kernel_precompute()
    _check_kernel(plan, inp, N)
    _check_backprojection(plan, inp, N, inp.rotations.shape[0], 64)
    b, _ = _check_solves(firm, plan, inp, N, _oracle_operator(plan, N, inp.workload.lam), 65)
    plan.close()
    # lambda read literally (1e-2 absolute, about 1e-9 of Ker(0) here): the system is singular to
    # FP32 working precision and plain CG does not reach 1e-5 within 3000 iterations
    lit = firm.Plan(N, inp.rotations, shifts=inp.shifts, ctf_group=inp.ctf_group, ctf_table=inp.ctf_table,
                    precision=1, lambda_relative=0)
    lit.kernel_precompute()
    _, rep = lit.cg_solve(b, inp.workload.lam, TOL, 3000)
    print(f"  literal lambda: status {rep['status']}, {rep['iters']} iterations, true rel res "
          f"{rep['true_rel_res']:.2e}", flush=True)
    assert rep["status"] == firm.FIRM_ERR_NOT_CONVERGED and rep["true_rel_res"] > TOL
    lit.close()


def test_uneven_workload_end_to_end_with_16bit_spectra(firm):
    inp = synth.make_inputs("uneven")
    N = inp.workload.N
    lam_rel = inp.workload.lam
    print(f"uneven: N={N} M={inp.rotations.shape[0]}", flush=True)
    plan = firm.Plan(N, inp.rotations, shifts=inp.shifts, ctf_group=inp.ctf_group, ctf_table=inp.ctf_table,
                     precision=1, lambda_relative=1)
    plan.kernel_precompute()
    _check_kernel(plan, inp, N)
    _check_backprojection(plan, inp, N, 60, 128)
    apply = _oracle_operator(plan, N, lam_rel)
    b, bh = _check_solves(firm, plan, inp, N, apply, 129)
    y_ref = apply(bh)
    for mode in (1, 2):
        p16 = firm.Plan(N, inp.rotations[:1], precision=1, lambda_relative=1, khat_bf16=mode)
        p16.kernel_set(plan.kernel_get())
        y = p16.apply_AtA(b, lam_rel).cpu().numpy()
        err = rel(y, y_ref)
        x, rep = p16.cg_solve(b, lam_rel, TOL, 3000)
        rr = float(np.linalg.norm(bh - apply(x.cpu().numpy().astype(np.float64))) / np.linalg.norm(bh))
        print(f"  16-bit spectrum {mode}: product rel err {err:.2e}; refined CG {rep['iters']} iterations, "
              f"oracle rel res {rr:.3e}", flush=True)
        assert err < 1e-3 and rep["status"] == 0 and rr <= TOL * 1.01
        p16.close()
    plan.close()
