"""Learned warm start for agf2_run: trajectories, training, evaluation.

Trajectories come from the method itself: for each seeded synthetic system
the GPU path builds the iteration-0 moments, runs AGF2 to self-consistency
from the cold start, and rebuilds the moments from the converged Green's
function. The network (agf2_mlp_*) learns, from per-orbital features of the
iteration-0 moments, the correction that takes them to the converged ones.
Training runs on the GPU through the library's forward, loss, backward and
Adam kernels; this module only schedules the calls (batches, steps, learning
rate) and moves tensors.

Evaluation: every held-out system is converged twice by agf2_run, from the
cold start and with the predicted correction as dm_init; the report gives
the iterations of both, their wall time and the differences of the converged
IP, EA and total energy (the cold-start result is the reference).

    python -m paper_2106_03508_amd.warmstart train --out params.npy
    python -m paper_2106_03508_amd.warmstart eval --params params.npy
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import agf2
from . import synthetic as syn

PARAMS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "warmstart_params.npy")

TRAIN_SET = dict(n=400, seed0=10000, nmo_lo=40, nmo_hi=160)
HELDOUT_SET = dict(n=24, seed0=20000, nmo_lo=60, nmo_hi=160)


def log(msg):
    print(f"# {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)


def load_params(path=PARAMS_PATH):
    return np.load(path, allow_pickle=False).astype(np.float32)


class System:
    """One synthetic system resident on the GPU (DF tensor, energies, the
    reference density and the core Hamiltonian that makes eps its Fock
    eigenvalues)."""

    def __init__(self, h, seed, nmo, nocc, naux):
        self.seed, self.N, self.nocc, self.naux = seed, nmo, nocc, naux
        d = h.device
        self.eps = torch.from_numpy(syn.orbital_energies(seed, nmo, nocc)).to(d)
        self.L = torch.from_numpy(syn.df_tensor(seed, nmo, naux, nocc)).to(d)
        D0 = torch.zeros(nmo, nmo, dtype=torch.float64, device=d)
        D0.diagonal()[:nocc] = 2.0
        self.hcore = agf2.agf2_fock_build(h, self.L, torch.diag(self.eps).contiguous(), D0, -1.0)
        self.eye = torch.eye(nmo, dtype=torch.float64, device=d)

    def moments(self, h, e_pole, u_pole, nocc_pole, prec="fp64"):
        out = h.empty(4, self.N, self.N)
        agf2.agf2_build_moments(h, self.L, e_pole, u_pole, nocc_pole, prec=prec,
                                out=tuple(out[k] for k in range(4)))
        return out

    def moments0(self, h, prec="fp64"):
        return self.moments(h, self.eps, self.eye, self.nocc, prec)

    def run(self, h, dm_init=None, prec="fp64", max_iter=40):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = agf2.agf2_run(h, self.L, self.hcore, self.eps, self.nocc,
                          agf2.run_opts(prec=prec, max_iter=max_iter), dm_init=dm_init)
        torch.cuda.synchronize()
        r["wall_s"] = time.perf_counter() - t0
        last = r["history"][-1]
        r.update(iterations=len(r["history"]) - 1, e_tot=last["e_tot"], ip=last["ip"],
                 ea=last["ea"], warm=r["history"][0]["warm"])
        return r


def trajectory(h, shape):
    """Training example of one system: features, scales, iteration-0 and
    converged moments, and the cold run's iteration count."""
    s = System(h, shape["seed"], shape["nmo"], shape["nocc"], shape["naux"])
    m0 = s.moments0(h)
    r = s.run(h)
    if not r["converged"]:
        return None
    mconv = s.moments(h, r["e_pole"], r["u_pole"], r["nocc_pole"])
    X, scale = agf2.agf2_mlp_features(h, s.eps, s.nocc, m0)
    return dict(N=s.N, X=X, scale=scale, m0=m0, mconv=mconv, iterations=r["iterations"],
                wall_s=r["wall_s"])


def generate(h, shapes, label):
    data = []
    t0 = time.perf_counter()
    for k, sh in enumerate(shapes):
        ex = trajectory(h, sh)
        if ex is not None:
            data.append(ex)
        if k % 20 == 19 or k == len(shapes) - 1:
            log(f"{label}: {k + 1}/{len(shapes)} systems converged "
                f"({time.perf_counter() - t0:.0f}s)")
    return data


def batch_loss(h, net, batch, train=True):
    """Forward (and backward) over a batch of examples stacked by rows;
    returns the summed loss as a device scalar."""
    X = torch.cat([ex["X"] for ex in batch]).contiguous()
    Y = agf2.agf2_mlp_forward(h, net, X)
    dY = torch.empty_like(Y)
    loss = torch.zeros(1, dtype=torch.float64, device=h.device)
    r0 = 0
    for ex in batch:
        N = ex["N"]
        agf2.agf2_mlp_loss_grad(h, Y[r0:r0 + N], ex["m0"], ex["mconv"], ex["scale"],
                                dY[r0:r0 + N], loss)
        r0 += N
    if train:
        agf2.agf2_mlp_backward(h, net, dY)
    return loss


def zero_loss(h, net_zero, data):
    """Loss of the zero correction (the cold start) on the same examples."""
    return sum(batch_loss(h, net_zero, data[i:i + 32], train=False).item()
               for i in range(0, len(data), 32))


def train(h, data, steps=6000, lr=3e-4, batch=8, seed=0, val_frac=0.1, init_seed=1):
    rng = np.random.default_rng(seed)
    idx = rng.permutation(len(data))
    nval = max(1, int(val_frac * len(data)))
    val = [data[i] for i in idx[:nval]]
    tr = [data[i] for i in idx[nval:]]
    net = agf2.Mlp(h, syn.mlp_init(init_seed))
    zero = agf2.Mlp(h, np.zeros(agf2.MLP_NPARAM, dtype=np.float32))
    base_tr, base_val = zero_loss(h, zero, tr), zero_loss(h, zero, val)
    zero.close()
    log(f"train {len(tr)} / validation {len(val)} systems; zero-correction loss "
        f"{base_tr / len(tr):.4e} / {base_val / len(val):.4e} per system")
    hist = []
    t0 = time.perf_counter()
    for step in range(1, steps + 1):
        pick = rng.choice(len(tr), size=min(batch, len(tr)), replace=False)
        loss = batch_loss(h, net, [tr[i] for i in pick])
        # cosine decay to 5% of the initial rate
        rate = lr * (0.05 + 0.95 * 0.5 * (1.0 + np.cos(np.pi * (step - 1) / steps)))
        agf2.agf2_mlp_adam_step(h, net, float(rate))
        if step % 500 == 0 or step == steps:
            vl = sum(batch_loss(h, net, val[i:i + 32], train=False).item()
                     for i in range(0, len(val), 32))
            hist.append(dict(step=step, train=loss.item() / len(pick), val=vl / len(val)))
            log(f"step {step}: batch loss {loss.item() / len(pick):.4e}, validation "
                f"{vl / len(val):.4e} ({vl / base_val:.3f} of the zero correction; "
                f"{time.perf_counter() - t0:.0f}s)")
    params = net.get_params()
    net.close()
    return params, dict(history=hist, zero_train=base_tr / len(tr), zero_val=base_val / len(val),
                        n_train=len(tr), n_val=len(val))


def evaluate(h, params, shapes, precs=("fp64",), exact=False):
    """Cold vs warm runs of each system. With exact=True the exact correction
    (converged minus iteration-0 moments) is also tried, as the bound a
    perfect predictor would reach."""
    net = agf2.Mlp(h, params)
    out = []
    for k, sh in enumerate(shapes):
        s = System(h, sh["seed"], sh["nmo"], sh["nocc"], sh["naux"])
        row = dict(seed=sh["seed"], nmo=sh["nmo"])
        cold = s.run(h)
        log(f"  nmo={sh['nmo']} cold fp64: {cold['iterations']} iterations, {cold['wall_s']:.1f}s")
        row["cold"] = {q: cold[q] for q in ("iterations", "wall_s", "e_tot", "ip", "ea",
                                            "converged")}
        m0 = s.moments0(h)
        t0 = time.perf_counter()
        dm = agf2.agf2_mlp_predict_correction(h, net, s.eps, s.nocc, m0)
        torch.cuda.synchronize()
        t_pred = time.perf_counter() - t0
        for prec in precs:
            w = s.run(h, dm_init=dm, prec=prec)
            log(f"  nmo={sh['nmo']} warm {prec}: {w['iterations']} iterations, "
                f"{w['wall_s']:.1f}s")
            row[f"warm_{prec}"] = dict(
                iterations=w["iterations"], wall_s=w["wall_s"] + t_pred, warm=w["warm"],
                converged=w["converged"], d_ip=w["ip"] - cold["ip"], d_ea=w["ea"] - cold["ea"],
                d_e=w["e_tot"] - cold["e_tot"])
            if prec != "fp64":
                c2 = s.run(h, prec=prec)
                log(f"  nmo={sh['nmo']} cold {prec}: {c2['iterations']} iterations, "
                    f"{c2['wall_s']:.1f}s")
                row[f"cold_{prec}"] = dict(
                    iterations=c2["iterations"], wall_s=c2["wall_s"],
                    d_ip=c2["ip"] - cold["ip"], d_ea=c2["ea"] - cold["ea"],
                    d_e=c2["e_tot"] - cold["e_tot"])
        if exact:
            mconv = s.moments(h, cold["e_pole"], cold["u_pole"], cold["nocc_pole"])
            ex = torch.from_numpy(mconv.cpu().numpy() - m0.cpu().numpy()).to(h.device)
            w = s.run(h, dm_init=ex)
            row["exact"] = dict(iterations=w["iterations"], d_ip=w["ip"] - cold["ip"],
                                d_ea=w["ea"] - cold["ea"], d_e=w["e_tot"] - cold["e_tot"])
        out.append(row)
        wf = row["warm_fp64"] if "warm_fp64" in row else row[f"warm_{precs[0]}"]
        log(f"eval {k + 1}/{len(shapes)} nmo={sh['nmo']}: cold {row['cold']['iterations']} it "
            f"({row['cold']['wall_s']:.1f}s), warm {wf['iterations']} it ({wf['wall_s']:.1f}s), "
            f"dIP {wf['d_ip']:.1e} dEA {wf['d_ea']:.1e}"
            + (f", exact {row['exact']['iterations']} it" if exact else ""))
    net.close()
    return out


def summarize(rows, prec="fp64"):
    key = f"warm_{prec}"
    cold = np.array([r["cold"]["iterations"] for r in rows])
    warm = np.array([r[key]["iterations"] for r in rows])
    tc = np.array([r["cold"]["wall_s"] for r in rows])
    tw = np.array([r[key]["wall_s"] for r in rows])
    dev = max(max(abs(r[key]["d_ip"]), abs(r[key]["d_ea"])) for r in rows)
    out = dict(systems=len(rows), cold_iterations=float(cold.mean()),
               warm_iterations=float(warm.mean()),
               iterations_saved=float((cold - warm).mean()),
               fewer=int((warm < cold).sum()), more=int((warm > cold).sum()),
               cold_wall_s=float(tc.sum()), warm_wall_s=float(tw.sum()),
               max_ipea_diff=float(dev),
               max_energy_diff=float(max(abs(r[key]["d_e"]) for r in rows)),
               all_warm_used=bool(all(r[key]["warm"] for r in rows)))
    if "exact" in rows[0]:
        out["exact_iterations"] = float(np.mean([r["exact"]["iterations"] for r in rows]))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--n-train", type=int, default=TRAIN_SET["n"])
    t.add_argument("--nmo", type=int, nargs=2, default=[TRAIN_SET["nmo_lo"], TRAIN_SET["nmo_hi"]])
    t.add_argument("--steps", type=int, default=6000)
    t.add_argument("--lr", type=float, default=3e-4)
    t.add_argument("--batch", type=int, default=8)
    t.add_argument("--out", default=PARAMS_PATH)
    t.add_argument("--n-eval", type=int, default=HELDOUT_SET["n"])
    t.add_argument("--eval-nmo", type=int, nargs=2,
                   default=[HELDOUT_SET["nmo_lo"], HELDOUT_SET["nmo_hi"]])
    e = sub.add_parser("eval")
    e.add_argument("--params", default=PARAMS_PATH)
    e.add_argument("--n-eval", type=int, default=HELDOUT_SET["n"])
    e.add_argument("--eval-nmo", type=int, nargs=2,
                   default=[HELDOUT_SET["nmo_lo"], HELDOUT_SET["nmo_hi"]])
    e.add_argument("--seed0", type=int, default=HELDOUT_SET["seed0"])
    e.add_argument("--precs", nargs="+", default=["fp64"])
    e.add_argument("--exact", action="store_true")
    args = ap.parse_args()

    h = agf2.Handle(0)
    report = {}
    if args.cmd == "train":
        shapes = syn.batch_shapes(args.n_train, TRAIN_SET["seed0"], *args.nmo)
        data = generate(h, shapes, "trajectories")
        report["trajectories"] = dict(
            systems=len(data), failed=len(shapes) - len(data),
            mean_cold_iterations=float(np.mean([d["iterations"] for d in data])),
            wall_s=float(sum(d["wall_s"] for d in data)))
        params, info = train(h, data, steps=args.steps, lr=args.lr, batch=args.batch)
        np.save(args.out, params)
        log(f"parameters written to {args.out}")
        report["training"] = info
        del data
        params_eval = params
    else:
        params_eval = load_params(args.params)
    if args.n_eval > 0:
        seed0 = HELDOUT_SET["seed0"] if args.cmd == "train" else args.seed0
        shapes = syn.batch_shapes(args.n_eval, seed0, *args.eval_nmo)
        precs = ["fp64"] if args.cmd == "train" else args.precs
        rows = evaluate(h, params_eval, shapes, precs=precs,
                        exact=(args.cmd == "eval" and args.exact))
        report["evaluation"] = {p: summarize(rows, p) for p in precs}
        report["rows"] = rows
    print(json.dumps(report), flush=True)


if __name__ == "__main__":
    main()
