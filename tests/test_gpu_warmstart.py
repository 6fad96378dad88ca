"""GPU checks of the learned warm start: network kernels against the FP64
reference, dose features against their definitions, dual-consistent restart."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import exact, features, mlp, wls

pytestmark = pytest.mark.gpu


def _close(got, ref, rtol, atol):
    err = np.abs(np.asarray(got, dtype=np.float64) - ref)
    bound = rtol * np.abs(ref) + atol
    assert np.all(err <= bound), f"worst ratio {np.max(err / bound):.3g}"


@pytest.mark.parametrize("F,H,B", [(15, 128, 2900), (3, 16, 1), (20, 64, 37)])
def test_mlp_forward_and_gradient_parity(F, H, B):
    import paper_2304_14568_amd as A
    rng = np.random.default_rng(F * 1000 + B)
    net = A.Mlp(F, H, seed=3)
    th = net.get_params().astype(np.float64)
    assert th.size == sum(int(np.prod(s)) for _, s in mlp.shapes(F, H))
    X = rng.normal(size=(B, F)).astype(np.float32)
    t = rng.uniform(0, 3, size=B).astype(np.float32)
    y, lr = net.forward(X)
    yr, lrr, _ = mlp.forward(th, X, F, H)
    _close(y, yr, 1e-4, 1e-5 * max(1.0, np.abs(yr).max()))
    assert abs(lr - lrr) <= 1e-4 * max(1.0, abs(lrr))
    L, g = net.loss_grad(X, t, target_log_rho=0.4, lam=0.5)
    Lr, gr = mlp.loss_and_grad(th, X, t, 0.4, 0.5, F, H)
    assert abs(L - Lr) <= 1e-4 * max(1.0, Lr)
    # fp32 products of length <= max(F, H, B): error relative to the largest gradient entry
    _close(g, gr, 1e-3, 1e-4 * max(1e-6, np.abs(gr).max()))


def test_mlp_adam_step_parity():
    import paper_2304_14568_amd as A
    rng = np.random.default_rng(5)
    F, H, B = 9, 32, 100
    net = A.Mlp(F, H, seed=1)
    th = net.get_params().astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    X = rng.normal(size=(B, F)).astype(np.float32)
    t = rng.uniform(0, 1, size=B).astype(np.float32)
    for k in range(1, 4):
        # each step takes the GPU gradient at the GPU parameters; the reference
        # applies the same update in float64
        _, g = net.loss_grad(X, t)
        net.adam_step(lr=1e-2)
        th, m, v = mlp.adam(th, g.astype(np.float64), m, v, k, lr=1e-2)
        _close(net.get_params(), th, 1e-5, 1e-6)


def test_mlp_bf16_inference_close_to_fp32():
    import paper_2304_14568_amd as A
    rng = np.random.default_rng(6)
    net = A.Mlp(15, 128, seed=2)
    X = rng.normal(size=(500, 15)).astype(np.float32)
    y32, lr32 = net.forward(X)
    y16, lr16 = net.forward(X, precision="bf16")
    # bf16 storage of the hidden activations: ~2^-8 relative per term
    assert np.max(np.abs(y16 - y32)) <= 2e-2 * max(1.0, np.abs(y32).max())
    yo, lro = mlp.forward(net.get_params().astype(np.float64), X, 15, 128)[:2]
    assert np.max(np.abs(y16 - yo)) <= 2e-2 * max(1.0, np.abs(yo).max())
    assert abs(lr16 - lro) <= 2e-2 * max(1.0, abs(lro))


def test_mlp_training_reduces_loss():
    import paper_2304_14568_amd as A
    rng = np.random.default_rng(7)
    F, B = 4, 256
    X = rng.normal(size=(B, F)).astype(np.float32)
    t = np.log1p(np.exp(X[:, 0] - 0.5 * X[:, 1])).astype(np.float32)
    net = A.Mlp(F, 32, seed=0)
    L0, _ = net.loss_grad(X, t, want_grad=False)
    for _ in range(300):
        net.loss_grad(X, t)
        net.adam_step(lr=3e-3)
    L1, _ = net.loss_grad(X, t, want_grad=False)
    assert L1 < 0.1 * L0


def test_spot_features_parity():
    import paper_2304_14568_amd as A
    P = synth.hn_small(2)
    W = wls.from_problem(P)
    names = P.meta["struct_names"]
    cls = np.array([1 if nm.startswith("target") else 2 if nm.startswith("oar") else 0 for nm in names],
                   dtype=np.uint8)
    vc = cls[P.struct_id]
    ref = features.spot_features(W, vc)
    with A.Solver(P) as S:
        got = S.spot_features(vc)
    # sums of <= m fp32 products per column; feature 6 is a ratio of two such sums
    _close(got, ref, 1e-4, 1e-6)


@pytest.mark.parametrize("xupdate", ["cg", "dense"])
def test_dual_consistent_warm_start_at_optimum(xupdate):
    """Restarting at x* with y_s = -grad f_s(x*) leaves every x-update at x*
    and the consensus step at x*: the stop rule holds within a few iterations."""
    import paper_2304_14568_amd as A
    P = synth.make_tiny(0)
    W = wls.from_problem(P)
    Hm, g0, _ = wls.quadratic_form(W)
    xs, _ = exact.active_set(W, H=Hm, g0=g0)
    fs = wls.objective(W, xs)
    with A.Solver(P, max_iter=3000, xupdate=xupdate) as S:
        zs0, info0, st0 = S.solve()
        it_zero = info0[0]["iter"]
        S.warm_start(0, xs, dual_init=True)
        zs, info, st = S.solve()
        assert st == 0
        assert info[0]["iter"] <= max(3, it_zero // 10), (info[0]["iter"], it_zero)
        assert abs(wls.objective(W, zs[0]) - fs) <= 1e-6 * fs
        # without the duals the restart at x* still converges to x*
        S.warm_start(0, xs, dual_init=False)
        zs, info, st = S.solve()
        assert abs(wls.objective(W, zs[0]) - fs) <= 1e-5 * fs


def test_trained_warm_start_on_a_held_out_patient():
    """The committed network on a patient outside its training seeds: its z0 is
    feasible and much better than zero, and the dual-consistent restart from it
    meets the acceptance rule (objective within 1e-5 of the zero-initialised solve)."""
    import paper_2304_14568_amd as A
    from paper_2304_14568_amd import warmstart as W
    P = synth.hn_full(3001)
    ws = W.WarmStart.load()
    with A.Solver(P, max_iter=3000) as S:
        z_ref, i_ref, _ = W.solve_zero(S)
        f_ref = i_ref["obj"]
        z0, rho = ws.predict(S, P)
        assert np.all(z0 >= P.lb) and np.all(z0 <= P.ub)
        assert S.objective(z0) < 0.5 * S.objective(np.zeros(P.n))
        assert rho > 0
        z_w, i_w, _, _, _, _ = W.solve_warm(S, P, ws, f_ref=f_ref)
        assert i_w["obj"] - f_ref <= 1e-5 * f_ref


def test_what_the_trained_network_gains_on_held_out_patients():
    """The measured effect of the committed network on four held-out patients
    (seeds 3000-3003, outside the training seeds), against zero-initialised
    ADMM-BB: iterations to 1e-5 of the zero-initialised objective and wall
    time, for the full warm start (z0 with dual-consistent duals and the
    predicted penalty) and for the penalty head alone.  Pinned result: the warm
    start reaches the same objective (acceptance rule) but saves no
    iterations, and features plus inference make it slower in wall time; the
    penalty head alone stays within a few iterations of zero initialisation."""
    import torch
    from paper_2304_14568_amd import warmstart as W
    rows = W.compare([3000, 3001, 3002, 3003], stream=torch.cuda.current_stream())
    for r in rows:
        print(f"[warm] seed {r['seed']}: iterations to 1e-5 zero {r['iters_zero']} warm {r['iters_warm']} "
              f"rho-only {r['iters_rho']} (x{r['rho_factor']:.2f}); time zero {r['s_zero'] * 1e3:.1f} ms "
              f"warm {r['s_warm'] * 1e3:.1f} ms rho-only {r['s_rho'] * 1e3:.1f} ms", flush=True)
        assert r["f_warm"] - r["f_ref"] <= 1e-5 * r["f_ref"]
        assert r["iters_zero"] is not None and r["iters_warm"] is not None and r["iters_rho"] is not None
    it_ratio = np.mean([r["iters_warm"] / r["iters_zero"] for r in rows])
    t_ratio = np.mean([r["s_warm"] / r["s_zero"] for r in rows])
    rho_ratio = np.mean([r["iters_rho"] / r["iters_zero"] for r in rows])
    print(f"[warm] mean ratios to zero initialisation: iterations {it_ratio:.3f}, time {t_ratio:.3f}, "
          f"penalty-only iterations {rho_ratio:.3f}", flush=True)
    assert 0.85 <= it_ratio <= 1.3
    assert t_ratio >= 1.0
    assert 0.7 <= rho_ratio <= 1.5
