"""Experiments of Sec. 3 on the synthetic head-and-neck-shaped workloads.

  scaling   total runtime of ADMM-BB (dense and CG x-updates) and PGD (dense
            form; --sparse-pgd adds the sparse form) versus the
            number of scenarios N = 1..13 of one patient (Sec. 3.3, the
            scenario-count study), plus the time to reach the 1e-5 relative
            objective gap against the oracle's exact minimum where stored.
  precision bf16 / fp16 values inside CG against fp32 and the oracle minimum
  plans     plan quality of ADMM-BB and PGD (Table 2 style criteria, DVH bands)
  pgd       the dense PGD alone on one patient (paper stop, fixed budget)
  batch     several patients of uneven size in one context (one launch per
            phase for all of them), bf16 values inside CG, a shift-lattice
            scenario set; each patient cross-checked against its own fp32
            solve.

  python -m paper_2304_14568_amd.experiments scaling --out scaling.json
  python -m paper_2304_14568_amd.experiments batch --patients 8 --scen 64 --out batch.json

Everything runs on the GPU through the library; the oracle is not used here
(the stored minima it wrote are read by `refdata` when present).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import Solver, refdata

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _sync():
    import torch
    torch.cuda.synchronize()


def _stored_fstar(name: str, digest: str):
    return refdata.fstar(name, digest)


def _admm_run(P, f_ref, xupdate: str, stream):
    t0 = time.perf_counter()
    S = Solver(P, xupdate=xupdate, max_iter=5000, stream=stream)
    _sync()
    setup_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    zs, info, st = S.solve()
    _sync()
    solve_s = time.perf_counter() - t0
    out = dict(setup_s=setup_s, solve_s=solve_s, total_s=setup_s + solve_s, iters=info[0]["iter"],
               obj=info[0]["obj"], status=int(st), xupdate=S.xupdate()[0])
    if f_ref is not None:
        out["final_gap"] = (info[0]["obj"] - f_ref) / f_ref
        k = next((t["iter"] for t in S.trace() if (t["obj"] - f_ref) / f_ref <= 1e-5), None)
        if k is not None:
            S.reset()
            _sync()
            t0 = time.perf_counter()
            S.iterate(k)
            _sync()
            out["iters_to_1e-5"] = k
            out["time_to_1e-5_s"] = time.perf_counter() - t0
    S.close()
    return out


def _pgd_run(P, f_ref, stream, form: str = "dense", max_doublings: int = 14):
    """PGD with the paper's stop rule, and the time to the 1e-5 gap.

    dense: the device-driven form on the packed sum of the Gram matrices;
    sparse: the host-driven form over the sparse matrices (every iteration
    scans every A_s, as in the paper).  The first iteration count that reaches
    the gap is found by doubling then bisection over fixed iteration budgets
    (the iterates repeat from run to run) and timed on its own (power
    iteration for the step included, set-up excluded, as for ADMM-BB)."""
    S = Solver(P, xupdate="dense" if form == "dense" else "cg", stream=stream)
    dense = 1 if form == "dense" else 0
    _sync()
    t0 = time.perf_counter()
    x, info, st = S.pgd(0, dense=dense)  # the paper's rule: relative objective change <= 1e-5
    solve_s = time.perf_counter() - t0
    out = dict(form=form, solve_s=solve_s, iters=info["iter"], obj=info["obj"], status=int(st))
    if f_ref is not None:
        out["final_gap"] = (info["obj"] - f_ref) / f_ref

        def gap_at(k):
            t0 = time.perf_counter()
            _, inf, _ = S.pgd(0, obj_rel_tol=0.0, max_iter=k, dense=dense)
            return (inf["obj"] - f_ref) / f_ref, time.perf_counter() - t0

        k, lo = 16, 0
        for _ in range(max_doublings):
            gap, dt = gap_at(k)
            if gap <= 1e-5:
                break
            lo, k = k, 2 * k
        else:
            S.close()
            return out
        hi = k
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if gap_at(mid)[0] <= 1e-5:
                hi = mid
            else:
                lo = mid
        gap, dt = gap_at(hi)
        out["iters_to_1e-5"] = hi
        out["time_to_1e-5_s"] = dt
    S.close()
    return out


def cmd_scaling(args):
    import torch
    import synth
    stream = torch.cuda.Stream()
    P_all = synth.hn_full(args.seed)
    rows = []
    cases = []
    for N in [int(v) for v in args.n.split(",") if v]:
        name = f"hn_full_s{args.seed}" if N == P_all.num_scen else f"hn_full_s{args.seed}_n{N}"
        cases.append((name, (lambda N: (lambda: P_all.subset(list(range(N)))))(N)))
    if args.lattice:
        # the smallest patient of the batch recipe with its 64-scenario shift lattice
        cases.append(("batch_s10_p2", lambda: synth.batch_patient(2, num=8, scen=64, seed=10)))
    for name, make in cases:
        P = make()
        N = P.num_scen
        f_ref = _stored_fstar(name, P.digest())
        row = dict(N=N, workload=name, m=P.m, n=P.n, nnz=P.nnz, f_star=f_ref)
        for xu in ("dense", "cg"):
            row[f"admm_{xu}"] = _admm_run(P, f_ref, xu, stream)
        if not args.no_pgd:
            row["pgd"] = _pgd_run(P, f_ref, stream, "dense")
            if args.sparse_pgd:
                row["pgd_sparse"] = _pgd_run(P, f_ref, stream, "sparse")
            ta, tp = row["admm_dense"].get("time_to_1e-5_s"), row["pgd"].get("time_to_1e-5_s")
            if ta and tp:
                row["pgd_over_admm_time_to_1e-5"] = tp / ta
            # the like-for-like pair: both methods over the sparse matrices,
            # every iteration scanning every A_s (the paper's setting)
            tc = row["admm_cg"].get("time_to_1e-5_s")
            tps = row.get("pgd_sparse", {}).get("time_to_1e-5_s")
            if tc and tps:
                row["sparse_pgd_over_admm_cg_time_to_1e-5"] = tps / tc
        rows.append(row)
        msg = f"[scaling] N={N} dense {row['admm_dense']['total_s']:.3f}s cg {row['admm_cg']['total_s']:.3f}s"
        if "pgd" in row:
            msg += f" pgd {row['pgd']['solve_s']:.3f}s ({row['pgd']['iters']} it)"
        if "pgd_over_admm_time_to_1e-5" in row:
            msg += f" pgd/admm to 1e-5 {row['pgd_over_admm_time_to_1e-5']:.1f}x"
        if "sparse_pgd_over_admm_cg_time_to_1e-5" in row:
            msg += f" sparse pgd/admm cg to 1e-5 {row['sparse_pgd_over_admm_cg_time_to_1e-5']:.1f}x"
        print(msg, flush=True)
    res = dict(workload=f"hn_full({args.seed}) restricted to its first N scenarios"
                        + ("; batch patient 2 (seed 10) with 64 lattice scenarios" if args.lattice else ""), rows=rows)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
    print(json.dumps(res), flush=True)


def _batch_patients(num: int, scen: int, seed: int):
    """Patients of uneven size from the head-and-neck generator (the batch
    recipe of synth.batch_params: body and target scales drawn per patient,
    a shift-lattice scenario set)."""
    import synth
    out = []
    for k in range(num):
        P = synth.batch_patient(k, num=num, scen=scen, seed=seed)
        out.append(P)
        print(f"[batch] patient {k}: m={P.m} n={P.n} nnz={P.nnz}", flush=True)
    return out


def cmd_batch(args):
    import torch
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    Ps = _batch_patients(args.patients, args.scen, args.seed)
    gen_s = time.perf_counter() - t0
    res = dict(patients=[dict(m=P.m, n=P.n, nnz=P.nnz) for P in Ps], scenarios=args.scen,
               total_nnz=int(sum(P.nnz for P in Ps)), generate_s=gen_s, precision=args.precision)
    t0 = time.perf_counter()
    S = Solver(Ps, xupdate=args.xupdate, precision=args.precision, max_iter=args.max_iter, stream=stream)
    _sync()
    res["setup_s"] = time.perf_counter() - t0
    res["xupdate"], res["dense_factor_ms"] = S.xupdate()
    print(f"[batch] set-up {res['setup_s']:.1f}s ({res['xupdate']} x-update), {res['total_nnz']} nonzeros",
          flush=True)
    S.iterate(2)
    S.reset()
    _sync()
    t0 = time.perf_counter()
    S.iterate(args.steps)
    _sync()
    res["iters_per_s"] = args.steps / (time.perf_counter() - t0)
    S.reset()
    _sync()
    t0 = time.perf_counter()
    zs, infos, st = S.solve()
    _sync()
    res["solve_s"] = time.perf_counter() - t0
    res["solve"] = [dict(iters=i["iter"], obj=i["obj"], status=i["status"]) for i in infos]
    print(f"[batch] {res['iters_per_s']:.1f} it/s, solve {res['solve_s']:.1f}s", flush=True)
    S.close()
    # cross-check: every patient alone, fp32 values
    checks = []
    for k, P in enumerate(Ps):
        S1 = Solver(P, xupdate="cg", precision="fp32", max_iter=args.max_iter, stream=stream)
        _sync()
        t0 = time.perf_counter()
        z1, i1, _ = S1.solve()
        _sync()
        t_single = time.perf_counter() - t0
        f_batch = S1.objective(zs[k])
        checks.append(dict(obj_single_fp32=i1[0]["obj"], obj_batch_at_fp32=f_batch,
                           rel_diff=(f_batch - i1[0]["obj"]) / i1[0]["obj"], single_fp32_cg_solve_s=t_single,
                           single_iters=i1[0]["iter"]))
        S1.close()
        print(f"[batch] patient {k}: batch {f_batch:.6f} vs single fp32 {i1[0]['obj']:.6f}", flush=True)
    res["cross_check"] = checks
    res["sum_single_fp32_cg_solve_s"] = float(sum(c["single_fp32_cg_solve_s"] for c in checks))
    res["batched_over_single_fp32_time_ratio"] = res["solve_s"] / res["sum_single_fp32_cg_solve_s"]
    # time to 1e-5: the first iteration at which every patient's objective is
    # within 1e-5 of its single-patient fp32 solve, then that many iterations
    # timed from zero
    S = Solver(Ps, xupdate=args.xupdate, precision=args.precision, max_iter=args.max_iter, stream=stream)
    S.solve()
    ks = []
    for k in range(len(Ps)):
        f_ref = checks[k]["obj_single_fp32"]
        ks.append(next((t["iter"] for t in S.trace(k) if (t["obj"] - f_ref) <= 1e-5 * abs(f_ref)), None))
    if all(v is not None for v in ks):
        K = max(ks)
        S.reset()
        _sync()
        t0 = time.perf_counter()
        S.iterate(K)
        _sync()
        res["iters_to_1e-5"] = ks
        res["time_to_1e-5_s"] = time.perf_counter() - t0
        print(f"[batch] every patient within 1e-5 of its fp32 solve after {K} iterations: "
              f"{res['time_to_1e-5_s']:.2f} s", flush=True)
    S.close()
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
    print(json.dumps(res), flush=True)


def cmd_precision(args):
    """The precision forms of the CG x-update (bf16 / fp16 values with per-row
    fp32 scales inside CG, fp32 residual every iteration) against fp32 and the
    stored oracle minimum: objective, spot intensities, and the dose metrics a
    planner reads (max target dose, max OAR dose over all scenarios)."""
    import torch
    import synth
    from .clinical import evaluate
    stream = torch.cuda.Stream()
    P = synth.hn_full(args.seed)
    rec, xstar = refdata.load(f"hn_full_s{args.seed}")
    if rec is None or rec["digest"] != P.digest():
        raise SystemExit("stored oracle reference missing or stale")
    fstar = rec["f_star"]
    names = P.meta["struct_names"]
    tg = [g for g, nm in enumerate(names) if nm.startswith("target")]
    og = [g for g, nm in enumerate(names) if nm.startswith("oar")]
    rows = []
    with Solver(P, xupdate="cg", stream=stream) as S0:
        ev0 = evaluate(S0, P, xstar)
    ref_tmax = float(np.nanmax(ev0["metrics"]["Dmax"][:, tg]))
    ref_omax = float(np.nanmax(ev0["metrics"]["Dmax"][:, og]))
    for prec in ("fp32", "bf16", "fp16"):
        with Solver(P, xupdate="cg", precision=prec, max_iter=3000, stream=stream) as S:
            t0 = time.perf_counter()
            zs, info, st = S.solve()
            _sync()
            dt = time.perf_counter() - t0
            z = zs[0]
            k_hit = next((t["iter"] for t in S.trace() if (t["obj"] - fstar) / fstar <= 1e-5), None)
            t_hit = None
            if k_hit is not None:
                S.reset()
                _sync()
                t0 = time.perf_counter()
                S.iterate(k_hit)
                _sync()
                t_hit = time.perf_counter() - t0
            ev = evaluate(S, P, z)
            f = S.objective(z)
        tmax = float(np.nanmax(ev["metrics"]["Dmax"][:, tg]))
        omax = float(np.nanmax(ev["metrics"]["Dmax"][:, og]))
        row = {"precision": prec, "iters": info[0]["iter"], "solve_s": dt, "iters_to_1e-5": k_hit,
               "time_to_1e-5_s": t_hit}
        row.update(obj_rel_err=(f - fstar) / fstar,
                   z_rel_err_l2=float(np.linalg.norm(z - xstar) / np.linalg.norm(xstar)),
                   max_target_dose_rel_err=(tmax - ref_tmax) / ref_tmax,
                   max_oar_dose_rel_err=(omax - ref_omax) / ref_omax)
        rows.append(row)
        print(f"[precision] {json.dumps(row)}", flush=True)
    t32 = rows[0]["time_to_1e-5_s"]
    for r in rows:
        r["time_to_1e-5_ratio_vs_fp32"] = (r["time_to_1e-5_s"] / t32) if (t32 and r["time_to_1e-5_s"]) else None
    res = dict(workload=f"hn_full({args.seed})", reference="oracle x*, f* (tests/golden)",
               ref_max_target_dose=ref_tmax, ref_max_oar_dose=ref_omax, rows=rows)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)


def cmd_plans(args):
    """Plan quality of ADMM-BB and PGD on the same patient, the way Sec. 3
    compares them: Table 2 style criteria over the scenarios and the DVH bands
    of the targets (band width = max - min over scenarios of the DVH)."""
    import torch
    import synth
    from .clinical import evaluate, criteria_table
    stream = torch.cuda.Stream()
    P = synth.hn_full(args.seed)
    out = {}
    with Solver(P, stream=stream, max_iter=3000) as S:
        t0 = time.perf_counter()
        zs, info, _ = S.solve()
        _sync()
        plans = {"admm_bb": (zs[0], time.perf_counter() - t0, info[0]["iter"])}
        t0 = time.perf_counter()
        x, pinfo, _ = S.pgd(0)
        plans["pgd_paper_stop"] = (x, time.perf_counter() - t0, pinfo["iter"])
        t0 = time.perf_counter()
        x2, pinfo2, _ = S.pgd(0, obj_rel_tol=0.0, max_iter=args.pgd_iters)
        plans[f"pgd_{args.pgd_iters}_iters"] = (x2, time.perf_counter() - t0, pinfo2["iter"])
        for name, (x, dt, it) in plans.items():
            ev = evaluate(S, P, x)
            f = S.objective(x)
            bands = {}
            for g, nm in enumerate(ev["names"]):
                if nm.startswith("target"):
                    bands[nm] = float(np.nanmax(ev["dvh_band_max"][g] - ev["dvh_band_min"][g]))
            out[name] = dict(obj=f, seconds=dt, iters=it, criteria=ev["criteria"], target_dvh_band_max_width=bands)
            print(f"[plans] {name}: f={f:.6f} {dt:.3f}s {it} it, target DVH band widths {bands}", flush=True)
            print(criteria_table(ev), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(out, fh, indent=1)


def cmd_pgd(args):
    """The dense PGD on one patient: the paper's stop rule, then a fixed budget
    of iterations (the form the scaling study times), with the per-iteration rate."""
    import torch
    import synth
    stream = torch.cuda.Stream()
    P = synth.hn_full(args.seed)
    with Solver(P, xupdate="dense", stream=stream) as S:
        S.pgd(0, obj_rel_tol=0.0, max_iter=10)  # warm-up
        _sync()
        t0 = time.perf_counter()
        x, info, st = S.pgd(0)
        t_stop = time.perf_counter() - t0
        t0 = time.perf_counter()
        x, info2, st2 = S.pgd(0, obj_rel_tol=0.0, max_iter=args.iters)
        t_fix = time.perf_counter() - t0
    out = dict(n=P.n, scenarios=P.num_scen, paper_stop=dict(iters=info["iter"], obj=info["obj"], s=t_stop),
               fixed=dict(iters=info2["iter"], obj=info2["obj"], s=t_fix, us_per_iter=1e6 * t_fix / max(1, info2["iter"])))
    print(json.dumps(out), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2304_14568_amd.experiments")
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("scaling")
    a.add_argument("--seed", type=int, default=0)
    a.add_argument("--n", default="1,2,3,4,5,6,7,8,9,10,11,12,13")
    a.add_argument("--no-pgd", action="store_true")
    a.add_argument("--sparse-pgd", action="store_true", help="also time PGD over the sparse matrices")
    a.add_argument("--lattice", action="store_true",
                   help="add the smallest batch patient with its 64-scenario shift lattice")
    a.add_argument("--out", default="")
    a = sub.add_parser("pgd")
    a.add_argument("--seed", type=int, default=0)
    a.add_argument("--iters", type=int, default=1000)
    a = sub.add_parser("plans")
    a.add_argument("--seed", type=int, default=0)
    a.add_argument("--pgd-iters", type=int, default=2048)
    a.add_argument("--out", default="")
    a = sub.add_parser("precision")
    a.add_argument("--seed", type=int, default=0)
    a.add_argument("--out", default="")
    a = sub.add_parser("batch")
    a.add_argument("--patients", type=int, default=8)
    a.add_argument("--scen", type=int, default=64)
    a.add_argument("--seed", type=int, default=10)
    a.add_argument("--precision", default="bf16", choices=["fp32", "bf16", "fp16"])
    a.add_argument("--xupdate", default="cg", choices=["auto", "cg", "dense"])
    a.add_argument("--steps", type=int, default=20)
    a.add_argument("--max-iter", type=int, default=1000)
    a.add_argument("--out", default="")
    args = ap.parse_args(argv)
    {"scaling": cmd_scaling, "batch": cmd_batch, "precision": cmd_precision, "plans": cmd_plans,
     "pgd": cmd_pgd}[args.cmd](args)


if __name__ == "__main__":
    main()
