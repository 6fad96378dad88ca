"""Learned warm start for ADMM-BB on head-and-neck-shaped patients.

Per spot j of a patient the network sees
  * geometry (8): energy-layer position within its beam (0..1), range / 100 mm,
    beam's-eye-view offsets u / 50 mm, v / 50 mm from the target centroid and
    their radius / 50 mm, beam one-hot (3 beams);
  * dose (7): target and organ-at-risk shares of the spot's dose over the
    scenarios, log dose mass and the single-spot ideal intensity, computed on
    the GPU by the library (admm_spot_features);
and predicts the spot intensity z0_j = zscale * y_j (y from the softplus head)
and, from the pooled hidden layer, log of a factor on the default penalty.
The solve restarts from (z0, rho) with the duals y_s = -grad f_s(z0) that make
z0 a fixed point of every x-update (admm_warm_start with dual_init = 1).

Acceptance rule: a warm-started solve counts only if its objective is within
1e-5 relative of the zero-initialised solve's objective; otherwise the
zero-initialised solve is used and the fallback is counted.

Command line (all steps on the GPU):
  python -m paper_2304_14568_amd.warmstart data  --seeds 1000:1128 --out ws_train_a.npz
  python -m paper_2304_14568_amd.warmstart train --data a.npz b.npz --out weights.npz
  python -m paper_2304_14568_amd.warmstart eval  --weights weights.npz --seeds 5000:5064
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import NUM_DOSE_FEATURES, Mlp, Solver

GEOM_FEATURES = 8
NUM_FEATURES = GEOM_FEATURES + NUM_DOSE_FEATURES
RHO_SCALES = (1.0, 0.5)
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "warmstart_hn.npz")


def voxel_class(P) -> np.ndarray:
    """0 other, 1 target, 2 organ at risk, per voxel (from the structure names)."""
    names = P.meta["struct_names"]
    cls = np.array([1 if nm.startswith("target") else 2 if nm.startswith("oar") else 0 for nm in names],
                   dtype=np.uint8)
    return cls[np.asarray(P.struct_id, dtype=np.int64)]


def geometric_features(P) -> np.ndarray:
    meta = P.meta
    beam = np.asarray(meta["spot_beam"], dtype=np.int64)
    uv = np.asarray(meta["spot_uv"], dtype=np.float64)
    R = np.asarray(meta["spot_range"], dtype=np.float64)
    nb = 3
    out = np.zeros((P.n, GEOM_FEATURES), dtype=np.float32)
    for b in range(nb):
        sel = beam == b
        if sel.any():
            lo, hi = R[sel].min(), R[sel].max()
            out[sel, 0] = (R[sel] - lo) / (hi - lo) if hi > lo else 0.5
    out[:, 1] = R / 100.0
    out[:, 2] = uv[:, 0] / 50.0
    out[:, 3] = uv[:, 1] / 50.0
    out[:, 4] = np.hypot(uv[:, 0], uv[:, 1]) / 50.0
    out[np.arange(P.n), 5 + np.clip(beam, 0, nb - 1)] = 1.0
    return out


def features(S: Solver, P, patient: int = 0) -> np.ndarray:
    return np.concatenate([geometric_features(P), S.spot_features(voxel_class(P), patient)], axis=1)


class WarmStart:
    """A trained network with its input standardisation and output scale."""

    def __init__(self, theta, hidden, feat_mean, feat_std, zscale, rho_clamp=4.0, stream=None):
        self.hidden = int(hidden)
        self.feat_mean = np.asarray(feat_mean, dtype=np.float32)
        self.feat_std = np.asarray(feat_std, dtype=np.float32)
        self.zscale = float(zscale)
        self.rho_clamp = float(rho_clamp)
        self.net = Mlp(NUM_FEATURES, self.hidden, stream=stream)
        self.net.set_params(np.asarray(theta, dtype=np.float32))

    @classmethod
    def load(cls, path: str = DEFAULT_WEIGHTS, stream=None) -> "WarmStart":
        with np.load(path, allow_pickle=False) as f:
            return cls(f["theta"], int(f["hidden"]), f["feat_mean"], f["feat_std"], float(f["zscale"]),
                       float(f["rho_clamp"]), stream=stream)

    def normalise(self, X):
        return ((X - self.feat_mean) / self.feat_std).astype(np.float32)

    def predict(self, S: Solver, P, patient: int = 0, precision: str = "bf16"):
        """Returns (z0, rho) for the patient: network intensities clipped to the
        box and the default penalty times the clamped predicted factor."""
        X = self.normalise(features(S, P, patient))
        y, lr = self.net.forward(X, precision=precision)
        z0 = np.clip(y.astype(np.float64) * self.zscale, P.lb, P.ub)
        fac = float(np.clip(np.exp(lr), 1.0 / self.rho_clamp, self.rho_clamp))
        return z0, fac * S.rho(patient)


def iters_to_gap(S: Solver, f_ref: float, rel: float = 1e-5, patient: int = 0):
    """First iteration (1-based) whose objective is within rel of f_ref, from the solve's trace."""
    for t in S.trace(patient):
        if t["obj"] - f_ref <= rel * abs(f_ref):
            return int(t["iter"])
    return None


def solve_zero(S: Solver, patient: int = 0):
    S.warm_start(patient, None, 0.0, dual_init=False)
    t0 = time.perf_counter()
    zs, info, st = S.solve()
    return zs[patient], info[patient], time.perf_counter() - t0


def solve_warm(S: Solver, P, ws: WarmStart, patient: int = 0, f_ref=None):
    """Warm-started solve; the time includes features and inference.  With f_ref,
    also returns the first iteration within 1e-5 of it (else None)."""
    rho0 = S.rho(patient)
    t0 = time.perf_counter()
    z0, rho = ws.predict(S, P, patient)
    S.warm_start(patient, z0, rho, dual_init=True)
    zs, info, st = S.solve()
    dt = time.perf_counter() - t0
    k_gap = iters_to_gap(S, f_ref, patient=patient) if f_ref is not None else None
    S.warm_start(patient, None, rho0, dual_init=False)  # restore the default penalty
    return zs[patient], info[patient], dt, z0, rho, k_gap


def solve_rho_only(S: Solver, P, ws: WarmStart, patient: int = 0, f_ref=None):
    """Zero-initialised solve with only the network's penalty (the rho head);
    the time includes features and inference.  Returns (z, info, seconds, rho,
    iterations to 1e-5 of f_ref or None)."""
    rho0 = S.rho(patient)
    t0 = time.perf_counter()
    _, rho = ws.predict(S, P, patient)
    S.warm_start(patient, None, rho, dual_init=False)
    zs, info, st = S.solve()
    dt = time.perf_counter() - t0
    k_gap = iters_to_gap(S, f_ref, patient=patient) if f_ref is not None else None
    S.warm_start(patient, None, rho0, dual_init=False)
    return zs[patient], info[patient], dt, rho, k_gap


def compare(seeds, ws: WarmStart = None, stream=None):
    """Zero-initialised, warm-started and penalty-only solves of the given
    held-out patients: iterations to 1e-5 of the zero-initialised objective
    and wall times (warm and penalty-only times include features and
    inference).  Returns one dict per patient."""
    import synth
    ws = ws or WarmStart.load(stream=stream)
    out = []
    for seed in seeds:
        P = synth.hn_full(seed)
        with Solver(P, max_iter=2000, stream=stream) as S:
            S.solve()  # first solve of a context: page in code and caches
            _, i_ref, t_ref = solve_zero(S)
            f_ref = i_ref["obj"]
            k_ref = iters_to_gap(S, f_ref)
            _, i_w, t_w, _, _, k_w = solve_warm(S, P, ws, f_ref=f_ref)
            _, i_r, t_r, rho, k_r = solve_rho_only(S, P, ws, f_ref=f_ref)
            out.append(dict(seed=seed, f_ref=f_ref, iters_zero=k_ref, iters_warm=k_w, iters_rho=k_r,
                            s_zero=t_ref, s_warm=t_w, s_rho=t_r, f_warm=i_w["obj"], f_rho=i_r["obj"],
                            rho_factor=rho / S.rho()))
    return out


# ----------------------------------------------------------------------------
# dataset, training, evaluation
# ----------------------------------------------------------------------------

def _seeds(spec: str):
    a, b = spec.split(":")
    return list(range(int(a), int(b)))


def _patients(seeds, workers: int = 2):
    import synth
    with ThreadPoolExecutor(max_workers=workers) as ex:
        futs = [ex.submit(synth.hn_full, s) for s in seeds[:workers]]
        for i, s in enumerate(seeds):
            P = futs[i].result()
            if i + workers < len(seeds):
                futs.append(ex.submit(synth.hn_full, seeds[i + workers]))
            futs[i] = None
            yield s, P


def cmd_data(args):
    rows = dict(seed=[], n=[], f_star=[], iters=[], rho0=[], best_scale=[], solve_s=[])
    X_all, z_all = [], []
    t_start = time.perf_counter()
    for k, (seed, P) in enumerate(_patients(_seeds(args.seeds))):
        with Solver(P, max_iter=2000) as S:
            X = features(S, P)
            rho0 = S.rho()
            res = []
            for sc in RHO_SCALES:
                S.warm_start(0, None, sc * rho0, dual_init=False)
                t0 = time.perf_counter()
                zs, info, st = S.solve()
                res.append((info[0]["iter"] if st == 0 else 10 ** 9, info[0]["obj"], zs[0], time.perf_counter() - t0))
            ibest = int(np.argmin([r[0] for r in res]))
            iz = int(np.argmin([r[1] for r in res]))  # label: the lowest objective reached
        X_all.append(X)
        z_all.append(res[iz][2].astype(np.float32))
        rows["seed"].append(seed)
        rows["n"].append(P.n)
        rows["f_star"].append(res[iz][1])
        rows["iters"].append([r[0] for r in res])
        rows["rho0"].append(rho0)
        rows["best_scale"].append(RHO_SCALES[ibest])
        rows["solve_s"].append(res[0][3])
        print(f"[data] {k + 1} seed {seed} n {P.n} iters {[r[0] for r in res]} best x{RHO_SCALES[ibest]} "
              f"{time.perf_counter() - t_start:.0f}s", flush=True)
    np.savez_compressed(args.out, X=np.concatenate(X_all), z=np.concatenate(z_all),
                        **{k: np.asarray(v) for k, v in rows.items()})


def _load_data(paths):
    parts = [np.load(p, allow_pickle=False) for p in paths]
    X = np.concatenate([p["X"] for p in parts])
    z = np.concatenate([p["z"] for p in parts])
    n = np.concatenate([p["n"] for p in parts])
    best = np.concatenate([p["best_scale"] for p in parts])
    off = np.concatenate([[0], np.cumsum(n)])
    return X, z, n, off, best


def cmd_train(args):
    X, z, n, off, best = _load_data(args.data)
    P = len(n)
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std = np.where(std > 1e-6, std, 1.0)
    Xn = ((X - mean) / std).astype(np.float32)
    zscale = float(args.zscale)
    t = (z / zscale).astype(np.float32)
    lrt = np.log(best).astype(np.float32)
    net = Mlp(NUM_FEATURES, args.hidden, seed=args.seed)
    rng = np.random.default_rng(args.seed)
    hold = max(1, P // 10)
    order = rng.permutation(P)
    val, tr = order[:hold], order[hold:]
    t0 = time.perf_counter()
    best_val, best_theta = np.inf, net.get_params()
    for ep in range(args.epochs):
        lr = args.lr * (0.5 * (1 + np.cos(np.pi * ep / args.epochs)))
        tot = 0.0
        for p in rng.permutation(tr):
            sl = slice(off[p], off[p + 1])
            L, _ = net.loss_grad(Xn[sl], t[sl], float(lrt[p]), args.lam, want_grad=True)
            net.adam_step(lr=max(lr, 1e-5))
            tot += L
        if ep % 10 == 9 or ep == args.epochs - 1:
            vl = sum(net.loss_grad(Xn[off[p]:off[p + 1]], t[off[p]:off[p + 1]], float(lrt[p]), args.lam,
                                   want_grad=False)[0] for p in val) / len(val)
            if vl < best_val:
                best_val, best_theta = vl, net.get_params()
            print(f"[train] epoch {ep + 1} train {tot / len(tr):.5f} val {vl:.5f} {time.perf_counter() - t0:.0f}s",
                  flush=True)
    np.savez(args.out, theta=best_theta, hidden=np.int64(args.hidden), feat_mean=mean.astype(np.float32),
             feat_std=std.astype(np.float32), zscale=np.float64(zscale), rho_clamp=np.float64(4.0),
             info=np.asarray(json.dumps({"patients": int(P), "val_loss": float(best_val), "epochs": args.epochs,
                                         "lr": args.lr, "lam": args.lam})))


def cmd_eval(args):
    ws = WarmStart.load(args.weights)
    out = []
    t_start = time.perf_counter()
    for k, (seed, P) in enumerate(_patients(_seeds(args.seeds))):
        with Solver(P, max_iter=2000) as S:
            S.solve()  # first solve of a context: page in code and caches
            z_ref, i_ref, t_ref = solve_zero(S, 0)
            f_ref = i_ref["obj"]
            k_ref = iters_to_gap(S, f_ref)
            z_w, i_w, t_w, z0, rho, k_w = solve_warm(S, P, ws, f_ref=f_ref)
            f_w = i_w["obj"]
            accept = (f_w - f_ref) <= 1e-5 * f_ref
            r = dict(seed=seed, n=P.n, f_zero=f_ref, f_warm=f_w, iters_zero=i_ref["iter"], iters_warm=i_w["iter"],
                     s_zero=t_ref, s_warm=t_w, accept=bool(accept), rho_factor=rho / S.rho(),
                     gap_iters_zero=k_ref, gap_iters_warm=k_w,
                     z0_rel_err=float(np.linalg.norm(z0 - z_ref) / max(1e-30, np.linalg.norm(z_ref))),
                     f_z0_rel=(S.objective(z0) - f_ref) / f_ref)
        out.append(r)
        print(f"[eval] {k + 1} seed {seed} iters {r['iters_zero']} -> {r['iters_warm']} (to 1e-5: {k_ref} -> {k_w}) "
              f"time {t_ref * 1e3:.0f} -> {t_w * 1e3:.0f} ms accept {accept} z0 err {r['z0_rel_err']:.3f} "
              f"{time.perf_counter() - t_start:.0f}s", flush=True)
    acc = [r for r in out if r["accept"]]
    summ = dict(patients=len(out), accepted=len(acc), fallbacks=len(out) - len(acc),
                mean_iters_zero=float(np.mean([r["iters_zero"] for r in out])),
                mean_iters_warm_used=float(np.mean([r["iters_warm"] if r["accept"] else r["iters_zero"]
                                                    for r in out])),
                mean_s_zero=float(np.mean([r["s_zero"] for r in out])),
                # a fallback costs the warm attempt plus the zero-initialised solve
                mean_s_warm_used=float(np.mean([r["s_warm"] + (0 if r["accept"] else r["s_zero"]) for r in out])),
                median_z0_rel_err=float(np.median([r["z0_rel_err"] for r in out])),
                median_f_z0_rel=float(np.median([r["f_z0_rel"] for r in out])),
                mean_gap_iters_zero=float(np.mean([r["gap_iters_zero"] or 0 for r in out])),
                mean_gap_iters_warm=float(np.mean([r["gap_iters_warm"] or 0 for r in out])))
    print("[eval] summary " + json.dumps(summ), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(dict(summary=summ, patients=out), f, indent=1)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2304_14568_amd.warmstart")
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("data")
    a.add_argument("--seeds", required=True)
    a.add_argument("--out", required=True)
    a = sub.add_parser("train")
    a.add_argument("--data", nargs="+", required=True)
    a.add_argument("--out", required=True)
    a.add_argument("--hidden", type=int, default=128)
    a.add_argument("--epochs", type=int, default=150)
    a.add_argument("--lr", type=float, default=2e-3)
    a.add_argument("--lam", type=float, default=0.05)
    a.add_argument("--zscale", type=float, default=0.1)
    a.add_argument("--seed", type=int, default=0)
    a = sub.add_parser("eval")
    a.add_argument("--weights", default=DEFAULT_WEIGHTS)
    a.add_argument("--seeds", required=True)
    a.add_argument("--out", default="")
    args = ap.parse_args(argv)
    {"data": cmd_data, "train": cmd_train, "eval": cmd_eval}[args.cmd](args)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
