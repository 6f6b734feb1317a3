"""Training and evaluation of the learned Fourier-diagonal preconditioner.

Data: kernels of the 'train' recipe (N = 64, M = 10,000 views per set, vMF concentration
kappa ~ U[0, 20] with 10% uniform views, 1..20 CTF groups), each reduced on the GPU to the
network input (the 32^3 pooled log spectrum, firm_kernel_features) and the target of the
Kaporin objective (the Fourier diagonal t of A*A + lambda, firm_chan_spectrum).  Training runs
Adam on the library's own forward/backward kernels; evaluation counts the CG and PCG
iterations to a relative residual of 1e-5 on held-out sets (plain CG, the learned diagonal and
the analytic 1 / t), all with FP64 iterative refinement (precision 1).

Usage:
  python -m paper_1307_5824_amd.train_precond --sets 2000 --held 200 --epochs 3 \\
      --out paper_1307_5824_amd/weights/pcnet_kaporin.npy
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "pcnet_kaporin.npy")
C = 32


def init_params(seed=0):
    """He-scaled weights in the library's layout (w1 b1 w2 b2 w3 b3 w4 b4); the last layer is
    zero, so the untrained network gives d = 1 / (pooled |K^| + lambda)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, (co, ci) in enumerate([(C, 1), (C, C), (C, C), (1, C)]):
        w = rng.standard_normal(co * ci * 27) * np.sqrt(2.0 / (ci * 27))
        if i == 3:
            w[:] = 0.0
        parts += [w, np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


def load_weights(path=DEFAULT_WEIGHTS):
    return np.load(path).astype(np.float32)


def make_set(firm, synth, index, lam_rel, keep_plan=False):
    """(features, t, Ker(0), plan or None) of training-recipe set `index` on the GPU."""
    inp = synth.make_inputs("train", set_index=index)
    N = inp.workload.N
    plan = firm.Plan(N, inp.rotations, ctf_group=inp.ctf_group, ctf_table=inp.ctf_table, lambda_relative=1,
                     precision=1)
    plan.kernel_precompute()
    feat = plan.kernel_features(lam_rel)
    t = plan.chan_spectrum(lam_rel)
    ker0 = float(plan.kernel_get()[N, N, N].item())
    if not keep_plan:
        plan.close()
        plan = None
    return feat, t, ker0, plan


def evaluate(firm, torch, net, held, lam_rel, tol=1e-5, max_iter=3000, seed=7):
    """CG / learned PCG / analytic PCG iterations and times on held-out sets."""
    rows = []
    g = torch.Generator(device="cuda").manual_seed(seed)
    for feat, t, ker0, plan in held:
        N = plan.N
        atb = torch.randn((N, N, N), device="cuda", generator=g)
        d = plan.precond_from_output(net.forward(feat[None]))
        out = {}
        for name, pc in (("cg", None), ("learned", d), ("chan", 1.0 / t)):
            _, rep = plan.cg_solve(atb, lam_rel, tol, max_iter, precond=pc)
            out[name] = (rep["iters"], rep["t_ms"], rep["true_rel_res"])
        rows.append(out)
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sets", type=int, default=2000)
    ap.add_argument("--held", type=int, default=200)
    ap.add_argument("--eval", type=int, default=20, help="held-out sets on which CG is run")
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lam-rel", type=float, default=1e-2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args(argv)

    import torch

    from paper_1307_5824_amd import firm, synth

    t0 = time.perf_counter()
    feats, ts, k0s = [], [], []
    for s in range(args.sets):
        f, t, k0, _ = make_set(firm, synth, s, args.lam_rel)
        feats.append(f)
        ts.append(t)
        k0s.append(k0)
        if (s + 1) % 200 == 0:
            print(f"built {s + 1} training sets ({time.perf_counter() - t0:.1f} s)", flush=True)
    feats = torch.stack(feats)
    ts = torch.stack(ts)
    k0s = np.array(k0s)
    held = [make_set(firm, synth, args.sets + s, args.lam_rel, keep_plan=s < args.eval) for s in range(args.held)]
    print(f"built {args.held} held-out sets ({time.perf_counter() - t0:.1f} s)", flush=True)
    held_feats = torch.stack([h[0] for h in held])
    held_ts = torch.stack([h[1] for h in held])
    held_k0 = np.array([h[2] for h in held])
    N = synth.WORKLOADS["train"].N

    net = firm.PCNet(max_batch=args.batch)
    net.set_params(init_params(args.seed))

    def held_loss():
        tot = 0.0
        for i in range(0, args.held, args.batch):
            j = min(args.held, i + args.batch)
            tot += net.loss_grad(held_feats[i:j], N, held_ts[i:j], ker0=held_k0[i:j], with_grad=False,
                                 objective="kaporin")[0] * (j - i)
        return tot / args.held

    hist = [{"epoch": 0, "held_loss": held_loss()}]
    print(f"epoch 0: held-out Kaporin loss {hist[-1]['held_loss']:.4f}", flush=True)
    rng = np.random.default_rng(args.seed)
    t1 = time.perf_counter()
    for ep in range(1, args.epochs + 1):
        order = rng.permutation(args.sets)
        tr = 0.0
        nb = 0
        for i in range(0, args.sets - args.batch + 1, args.batch):
            idx = torch.as_tensor(order[i:i + args.batch], device="cuda")
            tr += net.train_step(feats[idx].contiguous(), N, ts[idx].contiguous(), ker0=k0s[order[i:i + args.batch]],
                                 lr=args.lr, objective="kaporin")
            nb += 1
        hist.append({"epoch": ep, "train_loss": tr / max(nb, 1), "held_loss": held_loss()})
        print(f"epoch {ep}: train {hist[-1]['train_loss']:.4f} held-out {hist[-1]['held_loss']:.4f} "
              f"({time.perf_counter() - t1:.1f} s)", flush=True)
    rows = evaluate(firm, torch, net, [h for h in held if h[3] is not None], args.lam_rel)
    it = {k: [r[k][0] for r in rows] for k in ("cg", "learned", "chan")}
    ms = {k: [r[k][1] for r in rows] for k in ("cg", "learned", "chan")}
    summary = {"sets": args.sets, "held": args.held, "eval": len(rows), "epochs": args.epochs,
               "history": hist, "mean_iters": {k: float(np.mean(v)) for k, v in it.items()},
               "mean_ms": {k: float(np.mean(v)) for k, v in ms.items()},
               "learned_beats_cg": int(sum(a < b for a, b in zip(it["learned"], it["cg"])))}
    print(json.dumps(summary), flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, net.get_params())
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(summary, f, indent=1)
    return summary


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
