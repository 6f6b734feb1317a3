"""FIRM hot-path benchmark on one MI355X.

One step is one pass of the whole hot path over one synthetic data set already resident in
HBM: kernel precompute (gridding + FFTs + circulant spectrum), back-projection A*b, a plain CG
solve to the tolerance, the learned preconditioner's inference (features, network, Chan's
spectrum, diagonal), the learned-PCG solve to the same tolerance, and a block of back-to-back
A*A products.  The headline value is A*A products per second at N = 256 (HIP events around the
product block).  The JSON line also carries the time to the tolerance of plain CG and learned
PCG (and, timed once after the steps, PCG with T. Chan's analytic diagonal and with a constant
floor under it at the network's mean level), the precompute and back-projection times with their
gridding rates, the forward projection and step 1 on real-space images, the paper's
random-conical-tilt accuracy experiment (Fourier cross-resolution outside and inside the missing
cone), the roofline of the dominant FFT pass and the FP64 oracle timed on the host's cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PASS_NAMES = ["rows_i3_pad_fwd", "cols_i2_fwd", "mid_i1_fwd_mul_inv", "cols_i2_inv", "rows_i3_inv_crop"]


def pass_bytes(N):
    """Algorithmic HBM bytes of the five passes of one plain product (FP32 spectrum, half spectrum
    along axis 3: N + 1 complex columns; lambda x is added through the middle pass's multiplier,
    so the last pass reads only T1)."""
    H = N + 1
    x = 4 * N ** 3
    t1 = 8 * N * N * H
    t2 = 8 * N * 2 * N * H
    kh = 4 * 2 * N * 2 * N * H
    return [x + t1, t1 + t2, t2 + kh + t2, t2 + t1, t1 + x]


def source_sha():
    h = hashlib.sha256()
    for f in ("fft.hip", "fft_core.h"):
        with open(os.path.join(ROOT, "paper_1307_5824_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(pass_index):
    """HBM bytes per launch of one pass of the product, from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by the factors a plain device copy gives), if it was
    taken on the current FFT sources; else None."""
    path = os.path.join(ROOT, "profiles", "apply_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_sha") != source_sha():
        return None
    try:
        return float(d["passes"][pass_index]["bytes_per_launch"])
    except (KeyError, IndexError, TypeError):
        return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(N, synth, seed=0):
    """The FP64 oracle timed on all host cores (a bounded sample of the same work, about 20 s):
    * value: FP64 Toeplitz products per second at size N through the 2N circulant embedding
      (scipy FFTs on every core), with the rates at N/4 and N/2 beside it;
    * the small workload's full oracle (direct kernel sum, direct back-projection, 20 FP64 CG
      iterations on the Toeplitz product);
    * the direct kernel sum of eq. kernel per offset at size N over all the headline workload's
      sample points (oracle/direct.c on every core), and the full (2N-1)^3 kernel extrapolated
      from it (labelled as such);
    * the mid workload's FP64 CG to 1e-5, extrapolated from the time of one FP64 iteration times
      the iterations the GPU's FP64-refined CG needs there (238)."""
    import numpy as np

    from oracle import blobs, direct
    from oracle import firm as ofirm
    cores = os.cpu_count() or 1
    rng = np.random.default_rng(seed)
    rates = {}
    for n, reps in ((N // 4, 5), (N // 2, 3), (N, 2)):
        K = rng.standard_normal((2 * n - 1,) * 3)
        K = 0.5 * (K + K[::-1, ::-1, ::-1])
        T = ofirm.toeplitz_operator(K, workers=cores)
        x = rng.standard_normal((n, n, n))
        T(x)
        t0 = time.perf_counter()
        for _ in range(reps):
            y = T(x)
        rates[n] = reps / (time.perf_counter() - t0)
        del K, T, x, y
    # the mid workload's CG iteration: one product plus the vector updates, FP64
    n = N // 4
    K = rng.standard_normal((2 * n - 1,) * 3)
    K = 0.5 * (K + K[::-1, ::-1, ::-1])
    T = ofirm.toeplitz_operator(K, workers=cores)
    b = rng.standard_normal((n, n, n))
    t0 = time.perf_counter()
    ofirm.cg(lambda v: T(v) + 1.0 * v, b, iters=10)
    it_s = (time.perf_counter() - t0) / 10
    # the small workload end to end
    inp = synth.make_inputs("small")
    Ns = inp.workload.N
    t0 = time.perf_counter()
    V = blobs.sample_volume(Ns, inp.centers, inp.sigmas, inp.amps)
    bsl = ofirm.forward_project(V, inp.rotations)
    Ker = ofirm.kernel_direct(Ns, inp.rotations).real
    atb = ofirm.back_project(bsl, Ns, inp.rotations).real
    Ts = ofirm.toeplitz_operator(Ker, workers=cores)
    ofirm.cg(lambda v: Ts(v) + inp.workload.lam * v, atb, iters=20)
    c1_s = time.perf_counter() - t0
    # the direct kernel sum per offset over the headline workload's 5.1e9 sample points
    big = synth.make_inputs("large")
    offs = np.array([[-40, 25, 90]])
    t0 = time.perf_counter()
    direct.kernel_at(offs, N, big.rotations, big.ctf_group, big.ctf_table, nthreads=cores)
    per_off = (time.perf_counter() - t0) / len(offs)
    return {"value": round(rates[N], 4), "unit": "applies/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 Toeplitz products at N={N} through the 2N circulant embedding (scipy FFTs on "
                      f"{cores} threads, random even kernel), 2 timed",
            "cpu_model": cpu_model(),
            "applies_per_s": {str(k): round(v, 4) for k, v in rates.items()},
            "small_full_oracle_s": round(c1_s, 3),
            "direct_kernel_s_per_offset": round(per_off, 3),
            "direct_kernel_full_s_extrapolated": round(per_off * (2 * N - 1) ** 3, 0),
            "mid_cg_iteration_s": round(it_s, 5),
            "mid_cg_to_1e-5_s_extrapolated": round(it_s * 238, 3)}


def counter_workload(args, firm, synth, torch):
    """Products at the workload's N on a random even kernel, then one plain device copy of
    COPY_BYTES: the copy's FETCH_SIZE / WRITE_SIZE per byte calibrate the counters."""
    N = synth.WORKLOADS[args.workload].N
    R = [[1.0, 0, 0, 0, 1.0, 0, 0, 0, 1.0]]
    plan = firm.Plan(N, R)
    g = torch.Generator(device="cuda").manual_seed(1)
    K = torch.randn((2 * N,) * 3, device="cuda", generator=g)
    K = 0.5 * (K + torch.flip(K, dims=(0, 1, 2)).roll((1, 1, 1), dims=(0, 1, 2)))
    plan.kernel_set(K.contiguous())
    x = torch.randn((N, N, N), device="cuda", generator=g)
    y = torch.empty_like(x)
    for _ in range(args.apply_reps):
        plan.apply_AtA(x, 0.1, y)
    src = torch.ones(COPY_BYTES // 4, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"counter_workload": f"N={N}", "applies": args.apply_reps, "copy_bytes": COPY_BYTES}),
          flush=True)


def spread_workload(args, firm, synth, torch):
    """One kernel precompute and one back-projection of the workload's slices (for counter
    runs on the two gridding kernels)."""
    inp = synth.make_inputs(args.workload)
    wl = inp.workload
    plan = firm.Plan(wl.N, inp.rotations, shifts=inp.shifts, ctf_group=inp.ctf_group, ctf_table=inp.ctf_table)
    b = plan.synth_slices(inp.centers, inp.sigmas, inp.amps, snr=wl.snr, seed=wl.index + 1)
    plan.kernel_precompute()
    plan.backproject(b)
    torch.cuda.synchronize()
    print(json.dumps({"spread_workload": f"{args.workload}: N={wl.N} M={inp.rotations.shape[0]}"}), flush=True)


COPY_BYTES = 256 * 1024 * 1024


def rct_experiment(args, firm, synth, torch, net, res):
    import numpy as np
    inp = synth.make_inputs("rct")
    wl = inp.workload
    N = wl.N
    plan = firm.Plan(N, inp.rotations, shifts=inp.shifts, ctf_group=inp.ctf_group, ctf_table=inp.ctf_table,
                     precision=args.precision, lambda_relative=1)
    b = plan.synth_slices(inp.centers, inp.sigmas, inp.amps, snr=wl.snr, seed=wl.index + 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.kernel_precompute()
    atb = plan.backproject(b)
    del b
    d = plan.precond_from_output(net.forward(plan.kernel_features(wl.lam, res=res)[None])[0],
                                 plan.chan_spectrum(wl.lam))
    x, rep = plan.cg_solve(atb, wl.lam, args.tol, args.max_iter, precond=d)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cone = 90.0 - wl.tilt_deg
    f = plan.fsc(x, plan.synth_volume(inp.centers, inp.sigmas, inp.amps), cone_deg=cone)
    plan.close()

    def first_below(row, level=0.5):
        idx = np.nonzero(np.nan_to_num(row, nan=1.0) < level)[0]
        return int(idx[0] + 1) if idx.size else int(row.size + 1)
    return {"workload": f"rct: N={N}, M={wl.M}, conical tilt {wl.tilt_deg:g} deg, {wl.groups} CTF groups, "
                        f"SNR {wl.snr:g}, lambda={wl.lam:g} x Ker(0)",
            "reconstruction_s": round(wall, 3), "learned_pcg_iters": rep["iters"],
            "missing_cone_half_angle_deg": cone,
            "fcr_0.5_shell": {"all": first_below(f[0]), "outside_cone": first_below(f[1]),
                              "inside_cone": first_below(f[2])},
            "mean_fcr_shells_1_to_N/4": {k: round(float(np.nanmean(f[i, :N // 4])), 4)
                                         for i, k in enumerate(("all", "outside_cone", "inside_cone"))}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--max-iter", type=int, default=3000)
    ap.add_argument("--precision", type=int, default=1)
    ap.add_argument("--apply-reps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["all", "apply", "spread"], default="all",
                    help="apply: only the N^3 products on a random even kernel plus a 256 MiB device copy "
                         "(the workload of the hardware-counter runs and their calibration); spread: one "
                         "kernel precompute and one back-projection (counter runs on the gridding)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested); the multi-GPU layout is a "
              "design note, not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1307_5824_amd import firm, synth

    torch.cuda.set_device(0)
    if args.only == "apply":
        counter_workload(args, firm, synth, torch)
        return
    if args.only == "spread":
        spread_workload(args, firm, synth, torch)
        return
    inp = synth.make_inputs(args.workload)
    wl = inp.workload
    N = wl.N
    plan = firm.Plan(N, inp.rotations, shifts=inp.shifts, ctf_group=inp.ctf_group, ctf_table=inp.ctf_table,
                     precision=args.precision, lambda_relative=1)
    b = plan.synth_slices(inp.centers, inp.sigmas, inp.amps, snr=wl.snr, seed=wl.index + 1)
    torch.cuda.synchronize()

    def ev():
        return torch.cuda.Event(enable_timing=True)

    x_probe = torch.randn((N, N, N), device="cuda")
    y_probe = torch.empty_like(x_probe)
    from paper_1307_5824_amd import train_precond
    net = firm.PCNet(max_batch=1)
    net.set_params(train_precond.load_weights())
    state = {}
    res = firm.inference_res(N)   # the network's grid
    t_l = torch.empty((N, N, N), device="cuda")

    def step():
        e = [ev() for _ in range(7)]
        e[0].record()
        plan.kernel_precompute()
        e[1].record()
        atb = plan.backproject(b)
        e[2].record()
        x, rep = plan.cg_solve(atb, wl.lam, args.tol, args.max_iter)
        e[3].record()
        o = net.forward(plan.kernel_features(wl.lam, res=res)[None])[0]
        d = plan.precond_from_output(o, plan.chan_spectrum(wl.lam, out=t_l))
        e[4].record()
        _, rep_l = plan.cg_solve(atb, wl.lam, args.tol, args.max_iter, precond=d)
        e[5].record()
        for _ in range(args.apply_reps):
            plan.apply_AtA(x_probe, wl.lam, y_probe)
        e[6].record()
        torch.cuda.synchronize()
        state["atb"] = atb
        state["x"] = x
        state["o"] = o
        return [e[i].elapsed_time(e[i + 1]) for i in range(6)], (rep, rep_l)

    for i in range(args.warmup):
        ph, _ = step()
        print(f"warmup {i}: phases ms {[round(v, 1) for v in ph]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phases, reps = [], []
    for i in range(args.steps):
        ph, rep = step()
        phases.append(ph)
        reps.append(rep)
        print(f"step {i}: phases ms {[round(v, 1) for v in ph]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ph = np.mean(np.array(phases), axis=0)
    applies_per_s = args.apply_reps / (ph[5] / 1e3)

    # the analytic ablation: PCG with the inverse of T. Chan's circulant spectrum (one untimed call
    # first, as the steps' warmup does for the learned path)
    t_chan = plan.chan_spectrum(wl.lam)
    d_chan = torch.reciprocal(t_chan)       # buffers, and torch's first reciprocal, outside the timed region
    torch.cuda.synchronize()
    e = [ev() for _ in range(3)]
    e[0].record()
    torch.reciprocal(plan.chan_spectrum(wl.lam, out=t_chan), out=d_chan)
    e[1].record()
    _, rep_c = plan.cg_solve(state["atb"], wl.lam, args.tol, args.max_iter, precond=d_chan)
    e[2].record()
    torch.cuda.synchronize()
    chan_ms = [e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])]
    # the untrained network's form at the trained network's mean level: a constant floor under
    # Chan's spectrum (what the network's spatial variation adds is measured against it)
    ker0 = float(plan.kernel_get()[N, N, N].item())
    floor = float(torch.exp(state["o"].double().mean()).item())
    d_fl = torch.reciprocal(t_chan + floor * ker0)
    _, rep_f = plan.cg_solve(state["atb"], wl.lam, args.tol, args.max_iter, precond=d_fl)
    del d_fl

    # the forward projector on the reconstruction, and the data residual ||A x - b|| / ||b||
    # (slice by slice in blocks, so that no second full copy of b is formed)
    e = [ev() for _ in range(2)]
    e[0].record()
    bx = plan.forward_project(state["x"])
    e[1].record()
    torch.cuda.synchronize()
    fwd_ms = e[0].elapsed_time(e[1])
    num = den = 0.0
    for i in range(0, wl.M, 8192):
        j = min(wl.M, i + 8192)
        num += torch.linalg.norm(bx[i:j] - b[i:j]).double().item() ** 2
        den += torch.linalg.norm(b[i:j]).double().item() ** 2
    del bx
    data_res = (num / den) ** 0.5
    print(f"forward projection {fwd_ms:.1f} ms, data residual {data_res:.4f}", file=sys.stderr, flush=True)

    # the paper's accuracy experiment (section 4) on its geometry: a random conical tilt series at
    # 60 degrees (same sizes as the headline workload, 3 CTF groups, SNR 1), reconstructed with the
    # learned PCG, and the Fourier cross-resolution against the true volume outside and inside the
    # 30-degree missing cone (modified FCR)
    rct = rct_experiment(args, firm, synth, torch, net, res)
    print(f"rct: {rct}", file=sys.stderr, flush=True)

    # Step 1 from real-space images: the generator's images (projections of the same blobs at
    # the same views and shifts, pixel noise at the same SNR, no CTF) -> slices
    e = [ev() for _ in range(3)]
    e[0].record()
    imgs = plan.synth_images(inp.centers, inp.sigmas, inp.amps, snr=wl.snr, seed=wl.index + 2)
    e[1].record()
    b_img = plan.images_to_slices(imgs)
    e[2].record()
    torch.cuda.synchronize()
    synth_img_ms, img2sl_ms = e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])
    del imgs, b_img
    print(f"images: synth {synth_img_ms:.1f} ms, images_to_slices {img2sl_ms:.1f} ms", file=sys.stderr, flush=True)

    # the learned preconditioner at the size it was trained at: held-out sets of the N = 64
    # training recipe (the weights were fitted on sets 0 .. 1999), a random right-hand side,
    # the same tolerance; learned PCG includes the inference, Chan PCG its spectrum
    held0, nheld = 2000, 5
    lam64 = synth.WORKLOADS["train"].lam
    g64 = torch.Generator(device="cuda").manual_seed(64)
    t64 = {"cg": [], "learned_pcg": [], "chan_pcg": []}
    it64 = {k: [] for k in t64}
    st64 = 0
    for s in range(-1, nheld):   # s = -1: one untimed round (first launches at this size)
        feat, t64_, _, p64, _ = train_precond.make_set(firm, synth, held0 + max(s, 0), lam64, keep_plan=True)
        rhs = torch.randn((p64.N,) * 3, device="cuda", generator=g64)
        e = [ev() for _ in range(4)]
        e[0].record()
        _, r_cg = p64.cg_solve(rhs, lam64, args.tol, args.max_iter)
        e[1].record()
        d64 = p64.precond_from_output(net.forward(feat[None])[0], p64.chan_spectrum(lam64))
        _, r_l = p64.cg_solve(rhs, lam64, args.tol, args.max_iter, precond=d64)
        e[2].record()
        _, r_c = p64.cg_solve(rhs, lam64, args.tol, args.max_iter,
                              precond=torch.reciprocal(p64.chan_spectrum(lam64)))
        e[3].record()
        torch.cuda.synchronize()
        p64.close()
        if s < 0:
            continue
        for i, (k, r) in enumerate((("cg", r_cg), ("learned_pcg", r_l), ("chan_pcg", r_c))):
            t64[k].append(e[i].elapsed_time(e[i + 1]) / 1e3)
            it64[k].append(r["iters"])
            st64 = max(st64, r["status"])
    training_size = {
        "workload": f"train recipe: N=64, M=10000, held-out sets {held0}-{held0 + nheld - 1}, "
                    f"lambda={lam64:g} x Ker(0), random right-hand side",
        **{k: round(float(np.mean(v)), 5) for k, v in t64.items()},
        "iters": {k: round(float(np.mean(v)), 1) for k, v in it64.items()},
        "speedup_learned_vs_cg": round(float(np.mean(t64["cg"]) / np.mean(t64["learned_pcg"])), 3),
        "status": int(st64)}
    print(f"training size: {training_size}", file=sys.stderr, flush=True)

    # roofline of the dominant pass of the product, timed live with HIP events on the plan stream
    plan.apply_AtA_timed(x_probe, wl.lam, 20)   # untimed: the first block after other work runs slower
    pass_ms = plan.apply_AtA_timed(x_probe, wl.lam, 50)
    pb = pass_bytes(N)
    k = int(np.argmax(pass_ms))
    achieved = pb[k] / (pass_ms[k] / 1e3) / 1e9
    kernel_names = [f"k_rows_r2c<{2 * N}>", f"k_cols<{2 * N}> (i2 forward)", f"k_mid<{2 * N}>",
                    f"k_cols<{2 * N}> (i2 inverse)", f"k_rows_c2r<{2 * N}>"]
    traffic = measured_traffic(k) if N == 256 else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kernel_names[k], "bytes_per_launch": pb[k], "avg_launch_ms": round(pass_ms[k], 4),
                "passes_ms": [round(v, 4) for v in pass_ms],
                "apply_model_gbs": round(sum(pb) / (sum(pass_ms) / 1e3) / 1e9, 1)}

    # gridding rates (unit: a sample point of the half disk; the k = 0 samples are added in closed
    # form): each point adds W^3 terms to the LDS tile, one 64-bit integer atomic each (the A*b
    # spread adds its real and imaginary parts in two launches: 2 W^3).  The bound is the LDS
    # atomic rate: 9.1 conflict-free 64-bit adds per clock per CU (measured), 256 CUs, 2.4 GHz.
    # The phases include the grids' FFTs, about 1% of them
    W = 7
    npts = wl.M * (firm.firm_slice_points(N) - 1) // 2
    atomic_peak = 9.1 * 256 * 2.4e9
    gridding = {}
    for name, ms, per_pt in (("kernel_spread", ph[0], W ** 3), ("backprojection_spread", ph[1], 2 * W ** 3)):
        ups = npts * per_pt / (ms / 1e3)
        gridding[name] = {"points": npts, "points_per_s": float(f"{npts / (ms / 1e3):.4g}"),
                          "updates_per_point": per_pt, "updates_per_s": float(f"{ups:.4g}"),
                          "lds_atomic_peak_per_s": float(f"{atomic_peak:.4g}"),
                          "lds_atomic_bound_frac": round(ups / atomic_peak, 4)}

    out = {
        "metric": "A*A applies/s at N=256; time-to-1e-5 residual, learned-PCG vs plain CG",
        "value": round(applies_per_s, 2),
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: N={N}, {wl.blobs} Gaussian blobs, M={wl.M} projections, "
                               f"vMF kappa={wl.kappa} views, {wl.groups} CTF groups, SNR {wl.snr:.4g}, "
                               f"lambda={wl.lam:g} x Ker(0), tol {args.tol:g}",
                   "N": N, "M": wl.M, "precision": args.precision, "apply_reps_per_step": args.apply_reps},
        "time_to_tol_s": {
            "cg": round(ph[2] / 1e3, 4),
            "learned_pcg": round((ph[3] + ph[4]) / 1e3, 4),
            "learned_inference": round(ph[3] / 1e3, 4),
            "chan_pcg": round(sum(chan_ms) / 1e3, 4),
            "chan_spectrum": round(chan_ms[0] / 1e3, 4),
            "const_floor_pcg": round(rep_f["t_ms"] / 1e3, 4),
            "const_floor": round(floor, 5),
            "speedup_learned_vs_cg": round(ph[2] / (ph[3] + ph[4]), 3),
            "iters": {"cg": int(np.mean([r[0]["iters"] for r in reps])),
                      "learned_pcg": int(np.mean([r[1]["iters"] for r in reps])), "chan_pcg": rep_c["iters"],
                      "const_floor_pcg": rep_f["iters"]},
            "true_rel_res": {"cg": float(np.max([r[0]["true_rel_res"] for r in reps])),
                             "learned_pcg": float(np.max([r[1]["true_rel_res"] for r in reps])),
                             "chan_pcg": rep_c["true_rel_res"]},
            "status": int(max(max(r[0]["status"], r[1]["status"]) for r in reps) or rep_c["status"]),
            "at_training_size": training_size},
        "precompute_ms": round(ph[0], 2),
        "backproject_ms": round(ph[1], 2),
        "forward_project_ms": round(fwd_ms, 2),
        "data_rel_residual": round(data_res, 5),
        "images_to_slices_ms": round(img2sl_ms, 2),
        "gridding": gridding,
        "rct": rct,
        "synth_images_ms": round(synth_img_ms, 2),
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(N, synth)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
