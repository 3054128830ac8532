"""Learned coarse-grid correction for the 2D Gross-Pitaevskii workload.

A coarse run (512 intervals, h = 80/512) is corrected every 10 RK4 steps by the
3-layer convolutional network of nlse.Corrector, trained to match a 4x finer run
(2048 intervals) of the plain solver.  Everything numerical runs in the library's
HIP kernels: the fine and coarse 2SHOC-RK4 runs, the injection restriction, the
network's features, forward and backward passes and the Adam update.  Python only
orders the calls; PyTorch only holds device buffers.

Data: for each training seed, a fine trajectory (1..8 vortices at random positions,
1e-3 noise) is run to t = 20 with dt_f = dt_c / 16; every 160 fine steps (= 10 coarse
steps) its state is injected onto the coarse nodes (every 4th node).  A pair is
(coarse state after 10 coarse steps from snapshot j, snapshot j + 1).  The defaults
(200 training seeds, 80 seeded-random windows of the 315 per trajectory, 12000 Adam
steps) reproduce the committed weights.

Evaluation on held-out seeds: relative L2 at t = 20 on the 513^2 coarse nodes of
  plain runs at 512, 1024 and 1536 intervals and of the corrected 512 run, all
against the 2048 run; E(n) = C n^-p fitted through the plain runs gives the plain
resolution n* with E(n*) = E_learned, and the speedup T_plain(n*) / T_learned.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import nlse_inputs as I  # noqa: E402

from . import nlse as N  # noqa: E402

L_HALF, A_COEF, S_COEF, OMEGA = 40.0, 0.5, -1.0, 0.05
N_FINE, FACTOR, T_END, N_COARSE_STEPS, EVERY = 2048, 4, 20.0, 3150, 10
DT_C = T_END / N_COARSE_STEPS
DT_F = DT_C / (FACTOR * FACTOR)
WEIGHTS = os.path.join(HERE, "weights", "corrector_gp2d_512.npz")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fine_problem(seed, n=N_FINE, noise=1e-3):
    g = I.grid(2, n, -L_HALF, L_HALF)
    psi, V = I.gp2d_multivortex(g, omega=OMEGA, mu=1.0, noise=noise, seed=seed)
    return g, psi, V


def coarse_potential(n=N_FINE // FACTOR):
    g = I.grid(2, n, -L_HALF, L_HALF)
    x, y = g.coords()
    return I.harmonic_potential((x, y), OMEGA)


def _solver(n, V, prec="f32"):
    return N.Solver(2, n, 2 * L_HALF / n, A_COEF, S_COEF, V, prec=prec)


def _tuned(s):
    """Let the library pick the fastest kernel variant for this grid (all variants give
    bit-identical fields; the choice is cached per grid for the process).  Untimed."""
    s.autotune(reps=10)
    return s


def fine_trajectory(seed, snapshots=True, noise=1e-3, prec="f32"):
    """Run the fine problem of `seed` to T_END in precision `prec`; return the injected coarse
    snapshots [N_COARSE_STEPS/EVERY + 1, 513, 513] (complex64, on the GPU) and the run time.
    Training data use FP32 fine runs; the evaluation's reference run is FP64."""
    import torch
    g, psi, V = fine_problem(seed, noise=noise)
    s = _solver(N_FINE, V, prec)
    s.set_field(psi.astype(s.dtype))
    _tuned(s)
    nc = N_FINE // FACTOR + 1
    nsnap = N_COARSE_STEPS // EVERY
    buf = torch.empty((N_FINE + 1, N_FINE + 1), dtype=torch.complex64 if prec == "f32" else torch.complex128,
                      device="cuda")
    snaps = torch.empty((nsnap + 1, nc, nc), dtype=torch.complex64, device="cuda")
    chunk = EVERY * FACTOR * FACTOR
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(nsnap + 1):
        if snapshots or j == nsnap:
            s.get_field(buf)
            N.inject(buf, N_FINE, snaps[j], FACTOR)
        if j < nsnap:
            s.step(chunk, DT_F)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s.close()
    return snaps, el


def make_pairs(snaps, V):
    """Coarse predictions: 10 coarse steps from each snapshot; returns (pred, ref) tensors."""
    import torch
    nc = snaps.shape[-1]
    s = _solver(nc - 1, V)
    pred = torch.empty_like(snaps[:-1])
    for j in range(snaps.shape[0] - 1):
        s.set_field(snaps[j])
        s.step(EVERY, DT_C)
        s.get_field(pred[j])
    torch.cuda.synchronize()
    s.close()
    return pred, snaps[1:]


def rollout_pairs(seed, params, scale, V, windows, noise=1e-3):
    """On-policy pairs: the corrected coarse run of `seed` itself (10 coarse steps, correction,
    as in learned_run), paired window by window with the injected fine state at the window's
    end.  pred = the coarse state after the window's 10 steps (before its correction), ref =
    inject(fine) at that time; `windows` seeded-random windows are kept (all if 0)."""
    import torch
    snaps, el = fine_trajectory(seed, noise=noise)
    nc = snaps.shape[-1]
    nwin = snaps.shape[0] - 1
    keep = np.arange(nwin) if not (0 < windows < nwin) else np.sort(
        np.random.default_rng(seed + 7).choice(nwin, windows, replace=False))
    s = _solver(nc - 1, V)
    m = N.Corrector(nc, nc, max_batch=1, V=V)
    m.set_params(params, scale)
    s.set_field(snaps[0])
    pred = torch.empty((len(keep), nc, nc), dtype=torch.complex64, device="cuda")
    slot = {int(j): k for k, j in enumerate(keep)}
    for j in range(nwin):
        s.step(EVERY, DT_C)
        if j in slot:
            s.get_field(pred[slot[j]])
        m.apply(s)
    torch.cuda.synchronize()
    ref = snaps[torch.as_tensor(keep + 1, device=snaps.device)].clone()
    s.close()
    m.close()
    del snaps
    # windows where the corrected run has left the fine trajectory (non-finite, or farther from
    # it than half its norm) are no training input: their targets are off the states it visits
    # while it still tracks the fine run
    d = torch.linalg.vector_norm((pred - ref).reshape(len(keep), -1), dim=1)
    r = torch.linalg.vector_norm(ref.reshape(len(keep), -1), dim=1)
    ok = torch.isfinite(d) & (d <= 0.5 * r)
    if not bool(ok.all()):
        idx = torch.nonzero(ok).flatten()
        pred, ref = pred.index_select(0, idx), ref.index_select(0, idx)
    return (pred, ref), el


def residual_scale(pairs):
    """RMS of (ref - pred) over interior nodes of a few pairs (host-side statistic)."""
    pred, ref = pairs[0]
    idx = np.linspace(0, pred.shape[0] - 1, 8).astype(int)
    d = (ref[idx] - pred[idx]).cpu().numpy()[:, 1:-1, 1:-1]
    return float(np.sqrt(np.mean(d.real ** 2 + d.imag ** 2)))


def train(pairs, V, steps=3000, batch=4, lr=2e-3, seed=0, scale=None, init=None, smooth=2, augment=0.0):
    """Adam on the FP32 master weights; cosine-decayed learning rate.  Returns (params, scale, losses)."""
    import torch
    rng = np.random.default_rng(seed)
    nc = pairs[0][0].shape[-1]
    m = N.Corrector(nc, nc, max_batch=batch, V=V)
    if scale is None:
        scale = residual_scale(pairs)
    m.set_params(init if init is not None else initial_params(seed), scale)
    m.set_target_filter(smooth)
    m.set_augment(augment, seed)
    pool = [(t, j) for t in range(len(pairs)) for j in range(pairs[t][0].shape[0])]
    bp = torch.empty((batch, nc, nc), dtype=torch.complex64, device="cuda")
    br = torch.empty_like(bp)
    losses = []
    for it in range(steps):
        pick = rng.choice(len(pool), size=batch, replace=False)
        for b, k in enumerate(pick):
            t, j = pool[k]
            bp[b].copy_(pairs[t][0][j])
            br[b].copy_(pairs[t][1][j])
        lr_t = lr * 0.5 * (1 + math.cos(math.pi * it / steps))
        losses.append(m.train_step(bp, br, max(lr_t, lr * 0.02)))
        if it % 500 == 0:
            log(f"[train] step {it}: loss {losses[-1]:.4e}")
    params = m.get_params()
    m.close()
    return params, scale, losses


def initial_params(seed=0):
    """Seeded He-style initial weights in the library's parameter order (last layer small)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((32, 9, 8)) * math.sqrt(2.0 / 72)
    W2 = rng.standard_normal((32, 9, 32)) * math.sqrt(2.0 / 288)
    W3 = rng.standard_normal((2, 9, 32)) * 1e-3
    return np.concatenate([W1.ravel(), np.zeros(32), W2.ravel(), np.zeros(32), W3.ravel(), np.zeros(2)]).astype(
        np.float32)


def plain_run(seed, n, prec="f32", noise=1e-3):
    """Plain run at n intervals; returns (field at T_END on the 512 grid's nodes, run time in s, steps).
    When n divides the fine grid the initial field is the fine one injected onto n; otherwise it is
    the same seeded problem built on the n grid (same vortices, its own noise realisation)."""
    import torch
    if N_FINE % n == 0:
        f = N_FINE // n
        g, psi, V = fine_problem(seed, noise=noise)
        psi_n = np.ascontiguousarray(psi[::f, ::f]).astype(np.complex64)
        V_n = np.ascontiguousarray(V[::f, ::f])
    else:
        g, psi_n, V_n = fine_problem(seed, n=n, noise=noise)
        psi_n = psi_n.astype(np.complex64)
    s = _solver(n, V_n, prec)
    s.set_field(psi_n)
    _tuned(s)
    if n == N_FINE // FACTOR:
        nsteps, dt = N_COARSE_STEPS, DT_C
    else:
        k = s.max_dt()
        nsteps = math.ceil(T_END / (0.5 * k))
        dt = T_END / nsteps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(nsteps, dt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = s.get_field()
    s.close()
    r = n // (N_FINE // FACTOR)
    return out[::r, ::r].astype(np.complex128), el, nsteps


def learned_run(seed, params, scale, noise=1e-3):
    import torch
    g, psi, V = fine_problem(seed, noise=noise)
    nc = N_FINE // FACTOR
    Vc = np.ascontiguousarray(V[::FACTOR, ::FACTOR])
    s = _solver(nc, Vc)
    s.set_field(np.ascontiguousarray(psi[::FACTOR, ::FACTOR]).astype(np.complex64))
    _tuned(s)
    m = N.Corrector(nc + 1, nc + 1, max_batch=1, V=Vc)
    m.set_params(params, scale)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step_corrected(m, N_COARSE_STEPS, DT_C, EVERY)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = s.get_field().astype(np.complex128)
    s.close()
    m.close()
    return out, el


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def evaluate(params, scale, seeds, sizes=(512, 1024, 1536), damping=(1.0,), noise=1e-3):
    res = []
    for sd in seeds:
        snaps, t_fine = fine_trajectory(sd, snapshots=False, noise=noise, prec="f64")
        R = snaps[-1].cpu().numpy().astype(np.complex128)
        row = {"seed": sd, "t_fine_s": t_fine, "E": {}, "T": {}}
        for n in sizes:
            out, el, ns = plain_run(sd, n, noise=noise)
            row["E"][n], row["T"][n] = rel(out, R), el
        row["E_learned_damped"] = {}
        for al in damping:
            out, el = learned_run(sd, params, scale * al, noise=noise)
            row["E_learned_damped"][al] = rel(out, R)
        row["E_learned"], row["T_learned"] = row["E_learned_damped"][damping[0]], el
        log(f"[eval] seed {sd}: E_plain {row['E']}, E_learned {row['E_learned_damped']}, T {row['T']}, "
            f"T_learned {el:.3f}s, T_fine {t_fine:.2f}s")
        res.append(row)
    return res


def summarize(res, sizes=(512, 1024, 1536)):
    """Fit E(n) = C n^-p through the mean plain errors; equal-error resolution and speedups."""
    E = {n: float(np.mean([r["E"][n] for r in res])) for n in sizes}
    T = {n: float(np.mean([r["T"][n] for r in res])) for n in sizes}
    El = float(np.mean([r["E_learned"] for r in res]))
    Tl = float(np.mean([r["T_learned"] for r in res]))
    Tf = float(np.mean([r["t_fine_s"] for r in res]))
    ln, le = np.log(list(sizes)), np.log([E[n] for n in sizes])
    p, c = np.polyfit(ln, le, 1)
    p = -p
    n_star = float(np.exp((c - math.log(El)) / p)) if El > 0 else float("inf")
    lt = np.polyfit(ln, np.log([T[n] for n in sizes]), 1)
    t_star = float(np.exp(np.polyval(lt, math.log(n_star))))
    # Richardson estimate of the reference run's own distance from the converged solution: with
    # E(n) ~ C n^-p, |u_2048 - u_inf| ~ E(1024) 2^-p / (1 - 2^-p) (the fitted p, not the scheme's 4,
    # because the Thomas-Fermi kink limits convergence)
    n_half = N_FINE // 2
    e_ref = E[n_half] * 2.0 ** (-p) / (1.0 - 2.0 ** (-p)) if n_half in E else float("nan")
    gains = [r["E"][sizes[0]] / r["E_learned"] for r in res]
    return {"E_plain": E, "T_plain_s": T, "E_learned": El, "T_learned_s": Tl, "T_fine_s": Tf,
            "seeds": [r["seed"] for r in res], "gain_per_seed": gains, "gain_worst": float(min(gains)),
            "fit_order_p": float(p), "n_equal_error": n_star, "T_plain_at_equal_error_s": t_star,
            "speedup_vs_plain_equal_error": t_star / Tl, "speedup_vs_fine": Tf / Tl,
            "gain_E512_over_learned": E[sizes[0]] / El, "E_fine_run_richardson": float(e_ref)}


def main():
    ap = argparse.ArgumentParser(description="train and evaluate the learned coarse-grid corrector")
    ap.add_argument("--train-seeds", default="1000-1199")
    ap.add_argument("--val-seeds", default="8000")
    ap.add_argument("--test-seeds", default="9000-9003")
    ap.add_argument("--steps", type=int, default=12000)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--smooth", type=int, default=2, help="binomial target filter half-width (0: none)")
    ap.add_argument("--augment", type=float, default=0.0, help="training-input noise")
    ap.add_argument("--train-noise", type=float, default=1e-3, help="noise of the training trajectories")
    ap.add_argument("--windows", type=int, default=80,
                    help="keep this many seeded-random 10-step windows per training trajectory (0: all 315)")
    ap.add_argument("--damping", default="1.0,0.7,0.5", help="correction scales tried on the validation seeds")
    ap.add_argument("--rollout-rounds", type=int, default=0,
                    help="rounds of on-policy fine-tuning: pairs from the corrected coarse run itself")
    ap.add_argument("--rollout-steps", type=int, default=4000, help="Adam steps per rollout round")
    ap.add_argument("--init", default=None, help="start from these weights (skips the first training)")
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--report", default=None)
    args = ap.parse_args()
    rng_of = lambda s: list(range(int(s.split("-")[0]), int(s.split("-")[1]) + 1)) if "-" in s else [int(s)]
    train_seeds, val_seeds, test_seeds = rng_of(args.train_seeds), rng_of(args.val_seeds), rng_of(args.test_seeds)
    Vc = coarse_potential()
    pairs, t_data = [], 0.0
    for sd in (train_seeds if args.init is None else []):
        snaps, el = fine_trajectory(sd, noise=args.train_noise)
        pred, ref = make_pairs(snaps, Vc)
        if 0 < args.windows < pred.shape[0]:   # a seeded subset keeps 200 trajectories within HBM
            import torch
            keep = np.sort(np.random.default_rng(sd).choice(pred.shape[0], args.windows, replace=False))
            idx = torch.as_tensor(keep, device=pred.device)
            pred, ref = pred.index_select(0, idx), ref.index_select(0, idx)
        del snaps
        pairs.append((pred, ref))
        t_data += el
        log(f"[data] seed {sd}: fine run {el:.2f}s, {pairs[-1][0].shape[0]} pairs")
    t0 = time.perf_counter()
    if args.init is None:
        params, scale, losses = train(pairs, Vc, steps=args.steps, lr=args.lr, batch=args.batch, smooth=args.smooth,
                                      augment=args.augment)
    else:
        params, scale = load_weights(args.init)
        losses = [float("nan")]
    t_train = time.perf_counter() - t0
    del pairs
    # on-policy rounds: the corrected run's own states as inputs, the fine run as the target; a
    # round's weights are kept only if they lower the validation error
    rounds = []
    if args.rollout_rounds:
        best = float(np.mean([r["E_learned"] for r in evaluate(params, scale, val_seeds)]))
        log(f"[rollout] validation E_learned before: {best:.4e}")
    for rnd in range(args.rollout_rounds):
        rp = []
        for sd in train_seeds:
            pr, el = rollout_pairs(sd, params, scale, Vc, args.windows, noise=args.train_noise)
            if pr[0].shape[0]:
                rp.append(pr)
            t_data += el
            log(f"[rollout] round {rnd} seed {sd}: fine run {el:.2f}s, {pr[0].shape[0]} pairs")
        npairs = sum(p[0].shape[0] for p in rp)
        log(f"[rollout] round {rnd}: {npairs} on-policy pairs")
        if not rp:
            break
        t0 = time.perf_counter()
        cand, _, rl = train(rp, Vc, steps=args.rollout_steps, lr=args.lr * 0.25, batch=args.batch,
                            smooth=args.smooth, augment=args.augment, scale=scale, init=params, seed=rnd + 1)
        t_train += time.perf_counter() - t0
        del rp
        e = float(np.mean([r["E_learned"] for r in evaluate(cand, scale, val_seeds)]))
        rounds.append({"round": rnd, "pairs": npairs, "loss_first": rl[0], "loss_last100": float(np.mean(rl[-100:])),
                       "val_E_learned": e, "kept": bool(np.isfinite(e) and e < best)})
        log(f"[rollout] round {rnd}: validation E_learned {e:.4e} (best {best:.4e})")
        if not (np.isfinite(e) and e < best):
            break
        params, losses, best = cand, rl, e
    # the correction scale is chosen on validation seeds, never on the test seeds
    damp = tuple(float(v) for v in args.damping.split(","))
    val = evaluate(params, scale, val_seeds, damping=damp)
    mean_val = {a: float(np.mean([r["E_learned_damped"][a] for r in val])) for a in damp}
    alpha = min(mean_val, key=mean_val.get)
    log(f"[val] mean E_learned by damping {mean_val}; chosen {alpha}")
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.savez(args.out, params=params, scale=np.array(scale * alpha), train_seeds=np.array(train_seeds),
             smooth=np.array(args.smooth), steps=np.array(args.steps))
    res = evaluate(params, scale * alpha, test_seeds)
    summ = summarize(res)
    summ.update({"train_seeds": train_seeds, "val_seeds": val_seeds, "test_seeds": test_seeds,
                 "windows_per_trajectory": args.windows or N_COARSE_STEPS // EVERY,
                 "train_steps": args.steps, "smooth": args.smooth, "damping": alpha, "val_E_by_damping": mean_val,
                 "t_data_s": t_data, "t_train_s": t_train, "loss_first": losses[0],
                 "loss_last100": float(np.mean(losses[-100:])), "scale": scale * alpha,
                 "train_noise": args.train_noise, "rollout_rounds": args.rollout_rounds, "init": args.init,
                 "rollout": rounds})
    log(json.dumps(summ, indent=1, default=float))
    if args.report:
        json.dump({"summary": summ, "per_seed": res, "validation": val}, open(args.report, "w"), indent=1,
                  default=float)


def load_weights(path=WEIGHTS):
    z = np.load(path, allow_pickle=False)
    return z["params"].astype(np.float32), float(z["scale"])


if __name__ == "__main__":
    main()
