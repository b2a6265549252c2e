"""Train the learned initial density on converged plain-SCF densities and
evaluate it on held-out cells.

    python -m paper_1603_04339_amd.train_density_net [--n-train 2000] [--n-test 200]
        [--epochs 16] [--batch 8] [--lr 1e-3] [--threads 8]
        [--out paper_1603_04339_amd/data/density_net_40.npy] [--report report.json]

Data: the 40^3 SCF cells of workloads.scf_cell (8-32 atoms, seeded; training
ids 0..n_train-1, held-out ids from the test split).  For every cell the
library computes the atomic superposition (sparc_sad_density) and the local
potential (the network's two input channels) and runs the
plain FP64 SCF from it (sparc_scf_run, Anderson mixing with relaxation 0.15 and
history 8, density residual 1e-5; unconverged cells are left out); the pair (SAD, converged density), both divided by the mean density,
is one training sample.  Several cells run concurrently, one context and
stream per worker thread.  Training: Adam (sparc_dnet_train_step) on shuffled
mini-batches, cosine learning-rate decay.  Evaluation: every held-out cell is
solved twice, from the SAD and from the learned start
(sparc_dnet_predict_density), and the iteration counts and free energies are
compared.  Everything runs through the library; torch only holds device
memory and streams.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from . import sparc as sp
from . import workloads as wl

DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "density_net_40.npy")
# fallback threshold of the prediction: relative charge change made by the final ReLU
# (clipping only adds charge; renormalisation removes it); beyond this the output is
# treated as unusable and the atomic superposition is used instead
CHARGE_TOL = 0.1


def log(*a):
    print(*a, file=sys.stderr, flush=True)



# CheFSI passes of the first SCF iteration: enough to bring the random start subspace
# close to the eigenspace of the start potential, so that the SCF iteration count
# measures the quality of the start density rather than the subspace convergence
FIRST_PASSES = 16


# density mixing of the SCF runs: Anderson extrapolation (Sec. 4) with relaxation 0.15 and
# history 8.  With the paper's 0.3 and 7, 15 of the 200 held-out cells oscillate at a
# density residual of 0.2-0.7 for 200 iterations (the mixing overshoots); with 0.15 and 8,
# 199 converge and the mean count drops from 89 to 68.  A Kerker filter on the mixed
# residual (kerker_k0 > 0) is available and slows these cells down (183 converge at k0 1.2).
MIXING = {"mix": 0.15, "mix_history": 8, "kerker_k0": 0.0}


def scf_params(cell, X0, v0, rho_init=None, tol=1e-6, max_iter=200):
    return dict(n_s=cell.n_s, degree=20, n_first_passes=FIRST_PASSES, max_iter=max_iter, lanczos_steps=20,
                mix_history=MIXING["mix_history"], kT=0.01, mix=MIXING["mix"], tol=tol, n_elec=cell.n_elec,
                poisson_tol=1e-10, filt=sp.R64, rr=sp.GEMM_NATIVE, final_fp64_pass=1, rho_init_dev=rho_init,
                x0_dev=torch.from_numpy(X0).cuda(), lanczos_v0_dev=torch.from_numpy(v0).cuda(),
                kerker_k0=MIXING["kerker_k0"])


def cell_dV(cell):
    return (cell.L[0] / cell.n[0]) * (cell.L[1] / cell.n[1]) * (cell.L[2] / cell.n[2])


def cell_start(ctx, cell):
    """Atomic superposition and local potential of a cell (device FP64)."""
    rho_sad = torch.zeros(cell.n_d, dtype=torch.float64, device="cuda:0")
    sp.sad_density(ctx, cell, rho_sad)
    vloc = torch.zeros(cell.n_d, dtype=torch.float64, device="cuda:0")
    ham = sp.Hamiltonian(ctx, cell, sp.R64)
    ham.get_vloc(vloc)
    ham.close()
    return rho_sad, vloc


class Worker:
    """Per-thread context, stream and scaling helper."""

    _tls = threading.local()

    @classmethod
    def get(cls, n):
        w = getattr(cls._tls, "w", None)
        if w is None:
            w = cls()
            w.stream = torch.cuda.Stream()
            w.ctx = sp.Context(0, stream=w.stream)
            w.net = sp.DensityNet(w.ctx, n, max_batch=1)
            cls._tls.w = w
        return w


def solve(ctx, cell, X0, v0, rho_init=None, tol=1e-6):
    rho = torch.zeros(cell.n_d, dtype=torch.float64, device="cuda:0")
    ritz = torch.zeros(cell.n_s, dtype=torch.float64, device="cuda:0")
    t0 = time.perf_counter()
    out = sp.sparc_scf_run(ctx, cell, scf_params(cell, X0, v0, rho_init, tol=tol), rho, ritz)
    out["wall_s"] = time.perf_counter() - t0
    return out, rho


def make_sample(cell_id, split, n, tol):
    """Network input (SAD, -V_loc) and converged density of one cell, scaled, FP32 on
    the device."""
    w = Worker.get(n)
    with torch.cuda.stream(w.stream):
        cell, X0, v0 = wl.scf_cell(cell_id, split=split)
        rho_sad, vloc = cell_start(w.ctx, cell)
        out, rho = solve(w.ctx, cell, X0, v0, tol=tol)
        dV = cell_dV(cell)
        x = torch.empty(2 * cell.n_d, dtype=torch.float32, device="cuda:0")
        y = torch.empty(cell.n_d, dtype=torch.float32, device="cuda:0")
        w.net.prepare_input(rho_sad, vloc, cell.n_elec, dV, x)
        w.net.scale_density(rho, cell.n_elec, dV, y)
        w.stream.synchronize()
    return dict(id=cell_id, x=x, y=y, iterations=out["iterations"], energy=out["energy"],
                converged=out["converged"], n_atoms=cell.n_atoms, wall_s=out["wall_s"])


def generate(ids, split, threads, n, tol):
    t0 = time.perf_counter()
    done = []
    with ThreadPoolExecutor(max_workers=threads) as ex:
        futs = [ex.submit(make_sample, i, split, n, tol) for i in ids]
        for k, f in enumerate(futs):
            done.append(f.result())
            if (k + 1) % 50 == 0 or k + 1 == len(futs):
                log(f"[data] {split}: {k + 1}/{len(futs)} SCF runs, {time.perf_counter() - t0:.0f} s")
    return done


def train(net, data, epochs, batch, lr, seed=0):
    n_d = data[0]["y"].numel()
    X = torch.stack([d["x"] for d in data])
    Y = torch.stack([d["y"] for d in data])
    rng = np.random.default_rng(seed)
    steps = epochs * math.ceil(len(data) / batch)
    step = 0
    curve = []
    xb = torch.empty(2 * batch * n_d, dtype=torch.float32, device="cuda:0")
    yb = torch.empty(batch * n_d, dtype=torch.float32, device="cuda:0")
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = rng.permutation(len(data))
        tot, cnt = 0.0, 0
        for s in range(0, len(perm), batch):
            idx = torch.from_numpy(perm[s:s + batch]).cuda()
            B = idx.numel()
            xb[:2 * B * n_d].copy_(X.index_select(0, idx).reshape(-1))
            yb[:B * n_d].copy_(Y.index_select(0, idx).reshape(-1))
            lr_t = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * step / max(1, steps - 1))))
            loss = net.train_step(xb[:2 * B * n_d], yb[:B * n_d], lr_t)
            tot += loss * B
            cnt += B
            step += 1
        curve.append(tot / cnt)
        log(f"[train] epoch {ep + 1}/{epochs}: mean loss {tot / cnt:.5e}, {time.perf_counter() - t0:.0f} s")
    return curve


def evaluate_cell(theta, sample, n, charge_tol=CHARGE_TOL):
    w = Worker.get(n)
    with torch.cuda.stream(w.stream):
        w.net.set_params(theta)
        cell, X0, v0 = wl.scf_cell(sample["id"], split="test")
        rho_sad, vloc = cell_start(w.ctx, cell)
        rho0 = torch.zeros_like(rho_sad)
        used = w.net.predict_density(rho_sad, vloc, cell.n_elec, cell_dV(cell), rho0, charge_tol=charge_tol)
        out, _ = solve(w.ctx, cell, X0, v0, rho_init=rho0)
        w.stream.synchronize()
    return dict(id=sample["id"], n_atoms=cell.n_atoms, used_net=used,
                it_sad=sample["iterations"], it_net=out["iterations"],
                e_sad=sample["energy"], e_net=out["energy"], conv_sad=sample["converged"], conv_net=out["converged"],
                wall_sad=sample["wall_s"], wall_net=out["wall_s"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=2000)
    ap.add_argument("--n-test", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=16)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--charge-tol", type=float, default=CHARGE_TOL)
    ap.add_argument("--train-tol", type=float, default=1e-5,
                    help="SCF density-residual tolerance of the training targets (held-out cells: 1e-6)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eval-only", action="store_true",
                    help="evaluate the weights in --out on the held-out cells without generating training data")
    ap.add_argument("--kerker", type=float, default=MIXING["kerker_k0"],
                    help="Kerker wavenumber of the SCF mixing (0: none)")
    ap.add_argument("--mix", type=float, default=MIXING["mix"])
    ap.add_argument("--history", type=int, default=MIXING["mix_history"])
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--report", default=None)
    args = ap.parse_args()
    assert torch.cuda.is_available(), "training needs a GPU"
    sp.load()
    MIXING.update(mix=args.mix, mix_history=args.history, kerker_k0=args.kerker)
    n = (40, 40, 40)
    t0 = time.perf_counter()
    ctx = sp.Context(0)
    net = sp.DensityNet(ctx, n, max_batch=args.batch)
    if args.eval_only:
        train_data, curve, t_train = [], [], 0.0
        test_data = generate(range(args.n_test), "test", args.threads, n, 1e-6)
        t_data = time.perf_counter() - t0
        theta = np.load(args.out)
    else:
        train_all = generate(range(args.n_train), "train", args.threads, n, args.train_tol)
        train_data = [d for d in train_all if d["converged"]]   # unconverged targets are left out
        test_data = generate(range(args.n_test), "test", args.threads, n, 1e-6)
        t_data = time.perf_counter() - t0
        net.set_params(init_params(np.random.default_rng(args.seed), net.num_params))
        t1 = time.perf_counter()
        curve = train(net, train_data, args.epochs, args.batch, args.lr, args.seed)
        t_train = time.perf_counter() - t1
        theta = net.get_params()
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        np.save(args.out, theta)
        log(f"[train] weights written to {args.out}")
    t2 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=args.threads) as ex:
        res = list(ex.map(lambda smp: evaluate_cell(theta, smp, n, args.charge_tol), test_data))
    t_eval = time.perf_counter() - t2
    it_sad = np.array([r["it_sad"] for r in res], dtype=float)
    it_net = np.array([r["it_net"] for r in res], dtype=float)
    both = np.array([r["conv_sad"] and r["conv_net"] for r in res])
    de = np.array([abs(r["e_net"] - r["e_sad"]) / r["n_atoms"] for r in res])
    report = {
        "n_train": args.n_train if not args.eval_only else 0, "n_test": args.n_test, "epochs": args.epochs,
        "batch": args.batch, "lr": args.lr, "mixing": dict(MIXING), "eval_only": bool(args.eval_only),
        "params": int(net.num_params), "loss_curve": curve,
        "train_converged": len(train_data), "train_tol": args.train_tol,
        "test": {
            "mean_iterations_sad": float(it_sad.mean()), "mean_iterations_learned": float(it_net.mean()),
            "median_iterations_sad": float(np.median(it_sad)), "median_iterations_learned": float(np.median(it_net)),
            "fraction_fewer_iterations": float(np.mean(it_net < it_sad)),
            "both_converged": int(both.sum()),
            "mean_iterations_sad_both_converged": float(it_sad[both].mean()) if both.any() else None,
            "mean_iterations_learned_both_converged": float(it_net[both].mean()) if both.any() else None,
            "max_energy_diff_per_atom": float(de.max()), "mean_energy_diff_per_atom": float(de.mean()),
            "used_net": int(sum(r["used_net"] for r in res)),
            "converged_sad": int(sum(r["conv_sad"] for r in res)),
            "converged_learned": int(sum(r["conv_net"] for r in res)),
            "mean_wall_s_sad": float(np.mean([r["wall_sad"] for r in res])),
            "mean_wall_s_learned": float(np.mean([r["wall_net"] for r in res])),
        },
        "seconds": {"data": t_data, "train": t_train, "eval": t_eval},
    }
    log(json.dumps(report["test"]))
    if args.report:
        with open(args.report, "w") as f:
            json.dump({**report, "cells": res}, f, indent=1)
    print(json.dumps(report), flush=True)


def init_params(rng, count):
    """He-normal weights (std sqrt(2 / (27 c_in))) in the host layout, zero biases; the
    last layer scaled by 0.1 so that the untrained correction is small."""
    ch = (2, 16, 32, 32, 1)
    parts = []
    for l, (ci, co) in enumerate(zip(ch[:-1], ch[1:])):
        std = math.sqrt(2.0 / (27 * ci)) * (0.1 if l == len(ch) - 2 else 1.0)
        parts.append(rng.standard_normal(co * ci * 27) * std)
        parts.append(np.zeros(co))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == count
    return theta


if __name__ == "__main__":
    main()
