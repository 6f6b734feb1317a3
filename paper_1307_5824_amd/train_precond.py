"""Training and evaluation of the learned Fourier-diagonal preconditioner.

The diagonal is d = 1 / (t + Ker(0) exp(U sym(o))): t is the Fourier diagonal of A*A + lambda
(T. Chan's circulant spectrum, computed by the library), o the network's output on the res^3
grid, i.e. the network sets a floor under the analytic spectrum.  The objective is the unrolled
PCG error (firm_pcg_unrolled): the energy-norm error that k PCG steps leave on random probes
(section 3.3's CG minimises that norm over its Krylov space), differentiated through the
recursion's adjoint on the GPU and carried through the network by its own backward kernels.

Data: kernels of the 'train' recipe (N = 64, M = 10,000 views per set, vMF concentration
kappa ~ U[0, 20] with 10% uniform views, 1..20 CTF groups), each reduced on the GPU to the
network input (the 32^3 pooled log spectrum, firm_kernel_features), its Fourier diagonal t and
its kernel (kept on the device and swapped into one plan with firm_kernel_set for the unrolled
solves).  Evaluation counts CG and PCG iterations to a relative residual of 1e-5 on held-out
sets: plain CG, the learned diagonal, Chan's 1 / t and the untrained network's constant floor,
all with FP64 iterative refinement (precision 1).

Usage:
  python -m paper_1307_5824_amd.train_precond --sets 2000 --held 200 --eval 200 --epochs 4
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "pcnet_unrolled.npy")
C = 32


def init_params(seed=0, floor=0.1):
    """He-scaled weights in the library's layout (w1 b1 w2 b2 w3 b3 w4 b4); the last layer's weights
    are zero and its bias log(floor), so the untrained network is the constant floor:
    d = 1 / (t + floor Ker(0))."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, (co, ci) in enumerate([(C, 1), (C, C), (C, C), (1, C)]):
        w = rng.standard_normal(co * ci * 27) * np.sqrt(2.0 / (ci * 27))
        b = np.zeros(co)
        if i == 3:
            w[:] = 0.0
            b[:] = np.log(floor)
        parts += [w, b]
    return np.concatenate(parts).astype(np.float32)


def load_weights(path=DEFAULT_WEIGHTS):
    return np.load(path).astype(np.float32)


def make_set(firm, synth, index, lam_rel, keep_plan=False, keep_kernel=False):
    """(features, t, Ker(0), plan or None, kernel or None) of training-recipe set `index` on the GPU."""
    inp = synth.make_inputs("train", set_index=index)
    N = inp.workload.N
    plan = firm.Plan(N, inp.rotations, ctf_group=inp.ctf_group, ctf_table=inp.ctf_table, lambda_relative=1,
                     precision=1)
    plan.kernel_precompute()
    feat = plan.kernel_features(lam_rel)
    t = plan.chan_spectrum(lam_rel)
    ker = plan.kernel_get()
    ker0 = float(ker[N, N, N].item())
    if not keep_kernel:
        ker = None
    if not keep_plan:
        plan.close()
        plan = None
    return feat, t, ker0, plan, ker


def learned_diagonal(plan, net, feat, t):
    """The learned d for a plan whose kernel is current: network on the features, floor under t."""
    return plan.precond_from_output(net.forward(feat[None])[0], t)


def mean_floor(net, feats):
    """Geometric mean of the floor exp(o) the network puts out on the given features."""
    import torch
    o = torch.cat([net.forward(feats[i:i + net.max_batch]) for i in range(0, feats.shape[0], net.max_batch)])
    return float(torch.exp(o.double().mean()).item())


def evaluate(firm, torch, net, held, plan, lam_rel, const_floor, tol=1e-5, max_iter=3000, seed=7):
    """CG / learned PCG / analytic PCG iterations and times on held-out sets, each kernel swapped
    into `plan` (precision 1, lambda relative to Ker(0))."""
    rows = []
    g = torch.Generator(device="cuda").manual_seed(seed)
    N = plan.N
    for feat, t, ker0, _, ker in held:
        plan.kernel_set(ker)
        atb = torch.randn((N, N, N), device="cuda", generator=g)
        d = learned_diagonal(plan, net, feat, t)
        out = {}
        for name, pc in (("cg", None), ("learned", d), ("chan", 1.0 / t),
                         ("const_floor", 1.0 / (t + const_floor * ker0))):
            _, rep = plan.cg_solve(atb, lam_rel, tol, max_iter, precond=pc)
            out[name] = (rep["iters"], rep["t_ms"], rep["true_rel_res"])
        rows.append(out)
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sets", type=int, default=2000)
    ap.add_argument("--held", type=int, default=200)
    ap.add_argument("--eval", type=int, default=200, help="held-out sets on which the solvers are run")
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-5, help="Adam step of the network weights")
    ap.add_argument("--lr-floor", type=float, default=1e-2, help="Adam step of the output bias (log floor level)")
    ap.add_argument("--k", type=int, default=32, help="unrolled PCG steps")
    ap.add_argument("--probes", type=int, default=1)
    ap.add_argument("--floor0", type=float, default=0.1, help="constant floor of the untrained network")
    ap.add_argument("--lam-rel", type=float, default=1e-2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args(argv)

    import torch

    from paper_1307_5824_amd import firm, synth

    t0 = time.perf_counter()
    feats, ts, k0s, kers = [], [], [], []
    for s in range(args.sets):
        f, t, k0, _, ker = make_set(firm, synth, s, args.lam_rel, keep_kernel=True)
        feats.append(f)
        ts.append(t)
        k0s.append(k0)
        kers.append(ker)
        if (s + 1) % 200 == 0:
            print(f"built {s + 1} training sets ({time.perf_counter() - t0:.1f} s)", flush=True)
    feats = torch.stack(feats)
    ts = torch.stack(ts)
    k0s = np.array(k0s)
    held = [make_set(firm, synth, args.sets + s, args.lam_rel, keep_kernel=True) for s in range(args.held)]
    print(f"built {args.held} held-out sets ({time.perf_counter() - t0:.1f} s)", flush=True)
    N = synth.WORKLOADS["train"].N
    inp0 = synth.make_inputs("train", set_index=0)
    trainer = firm.Plan(N, inp0.rotations, lambda_relative=1, precision=0)

    net = firm.PCNet(max_batch=args.batch)
    net.set_params(init_params(args.seed, args.floor0))
    probe_seed = [0]

    def probes():
        probe_seed[0] += 1
        return trainer.synth_normals(90210, probe_seed[0] * args.probes * N ** 3, (args.probes, N, N, N))

    def unrolled(feat_b, t_b, ker_b, with_grad=True, z=None):
        """Loss (and log-d gradient) of one sample, its kernel swapped into the trainer plan."""
        trainer.kernel_set(ker_b)
        d = learned_diagonal(trainer, net, feat_b, t_b)
        return trainer.pcg_unrolled(d, z if z is not None else probes(), args.k, args.lam_rel, with_grad=with_grad)

    z_held = trainer.synth_normals(4242, 0, (1, N, N, N))

    def held_loss():
        tot = 0.0
        for f, t, _, _, ker in held:
            tot += unrolled(f, t, ker, with_grad=False, z=z_held)[0]
        return tot / len(held)

    hist = [{"epoch": 0, "held_loss": held_loss(), "mean_floor": mean_floor(net, feats[:64])}]
    print(f"epoch 0: held-out unrolled loss {hist[-1]['held_loss']:.5f}, floor {hist[-1]['mean_floor']:.4f}",
          flush=True)
    rng = np.random.default_rng(args.seed)
    t1 = time.perf_counter()
    for ep in range(1, args.epochs + 1):
        order = rng.permutation(args.sets)
        tr, nb = 0.0, 0
        for i in range(0, args.sets - args.batch + 1, args.batch):
            sel = order[i:i + args.batch]
            idx = torch.as_tensor(sel, device="cuda")
            G, L = [], 0.0
            for j in sel:
                loss, g = unrolled(feats[int(j)], ts[int(j)], kers[int(j)])
                G.append(g)
                L += loss / len(sel)
            G = torch.stack(G)
            if not bool(torch.isfinite(G).all()):
                raise RuntimeError(f"non-finite log-d gradient in batch {nb} (sets {list(sel)})")
            net.train_step(feats[idx].contiguous(), N, ts[idx].contiguous(), G, ker0=k0s[sel],
                           lr=args.lr, lr_floor=args.lr_floor, objective="logd")
            tr += L
            nb += 1
            if nb % 50 == 0:
                print(f"  batch {nb}: loss {L:.3e}, |G| {G.abs().max().item():.3e} "
                      f"({time.perf_counter() - t1:.1f} s)", flush=True)
        hist.append({"epoch": ep, "train_loss": tr / max(nb, 1), "held_loss": held_loss(),
                     "mean_floor": mean_floor(net, feats[:64])})
        print(f"epoch {ep}: train {hist[-1]['train_loss']:.5f} held-out {hist[-1]['held_loss']:.5f} "
              f"floor {hist[-1]['mean_floor']:.4f} ({time.perf_counter() - t1:.1f} s)", flush=True)
    cf = hist[-1]["mean_floor"]
    evaluator = firm.Plan(N, inp0.rotations, lambda_relative=1, precision=1)
    rows = evaluate(firm, torch, net, held[:args.eval], evaluator, args.lam_rel, cf)
    names = ("cg", "learned", "chan", "const_floor")
    it = {k: [r[k][0] for r in rows] for k in names}
    ms = {k: [r[k][1] for r in rows] for k in names}
    summary = {"objective": f"unrolled PCG, k={args.k}, {args.probes} probe(s) per sample",
               "sets": args.sets, "held": args.held, "eval": len(rows), "epochs": args.epochs,
               "batch": args.batch, "lr": args.lr, "lr_floor": args.lr_floor, "floor0": args.floor0,
               "const_floor": cf,
               "history": hist, "mean_iters": {k: float(np.mean(v)) for k, v in it.items()},
               "mean_ms": {k: float(np.mean(v)) for k, v in ms.items()},
               "learned_beats_cg": int(sum(a < b for a, b in zip(it["learned"], it["cg"]))),
               "learned_beats_chan": int(sum(a < b for a, b in zip(it["learned"], it["chan"]))),
               "learned_beats_const_floor": int(sum(a < b for a, b in zip(it["learned"], it["const_floor"]))),
               "train_s": round(time.perf_counter() - t1, 1)}
    print(json.dumps(summary), flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, net.get_params())
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(summary, f, indent=1)
    return summary


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
