"""End to end: the learned warm start on a small portfolio family.

Labels are cold batched rAPDHG solves at relKKT 1e-8; the MLP is trained by the
library's own forward/backward/Adam kernels; held-out instances are solved to
relKKT 1e-6 from the predicted point (kept only if its relKKT beats the cold
start's) and from zeros.  Every warm-started result must meet the same
termination test as the cold one; the network must predict the held-out
solutions better than their training mean and cut iterations against the cold
start; against a constant start (the training-mean solution) its iteration count
is equal within the measured 5 %.
"""
import numpy as np
import pytest

import qpgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    from paper_2311_07710_amd import warmstart
    return warmstart


def test_learned_warm_start_gain(ws):
    from paper_2311_07710_amd import Settings
    fam = qpgen.portfolio_family(seed=5, n_assets=400, k=20, count=1400)
    n, m = fam.base.n, fam.base.m
    tr, te = np.arange(1200), np.arange(1200, 1400)
    nA, nQ = ws.family_norms(fam)
    with ws.BatchSolver(fam.batch(np.arange(3)), Settings()) as b:
        a3, q3 = b.norms()
    # the family shares A and Q: batched power iteration agrees with the single one
    assert np.allclose(a3, nA, rtol=1e-3) and np.allclose(q3, nQ, rtol=1e-3)
    X, Y, res, t_lab = ws.solve_family(fam, tr, Settings(eps=1e-8), chunk=512,
                                       log=lambda s: print(s, flush=True))
    assert all(r["status"] == 0 for r in res)
    omega = np.array([r["omega"] for r in res])
    model = ws.train(ws.features(fam, tr), ws.targets(X, Y, omega), n, m, hidden=(256, 256),
                     epochs=60, batch=128, lr=1e-3, seed=0)
    assert model.history[-1] < 0.5 * model.history[0]
    x0, y0, w0 = model.predict(ws.features(fam, te))
    # held-out solutions (1e-8): the network must predict them better than their mean
    Xt, Yt, rt_, _ = ws.solve_family(fam, te, Settings(eps=1e-8))
    zt = np.hstack([Xt, Yt])
    zp = np.hstack([x0, y0])
    zm = np.tile(np.hstack([X.mean(axis=0), Y.mean(axis=0)]), (te.size, 1))
    err_l = np.mean(np.sum((zp - zt) ** 2, axis=1))
    err_m = np.mean(np.sum((zm - zt) ** 2, axis=1))
    _, _, cold, t_cold = ws.solve_family(fam, te, Settings(eps=1e-6))
    xw, yw, warm, t_warm = ws.solve_family(fam, te, Settings(eps=1e-6), x0=x0, y0=y0, omega0=w0)
    xm = np.tile(X.mean(axis=0), (te.size, 1))
    ym = np.tile(Y.mean(axis=0), (te.size, 1))
    gm = np.full(te.size, np.exp(np.log(omega).mean()))
    _, _, meanst, _ = ws.solve_family(fam, te, Settings(eps=1e-6), x0=xm, y0=ym, omega0=gm)
    _, _, wonly, _ = ws.solve_family(fam, te, Settings(eps=1e-6), omega0=w0)
    it = lambda rs: np.array([r["iterations"] for r in rs], dtype=float)  # noqa: E731
    print(f"held-out squared error: learned {err_l:.3e}, mean solution {err_m:.3e} | "
          f"cold {it(cold).mean():.0f} it ({t_cold:.3f}s) | predicted omega only "
          f"{it(wonly).mean():.0f} it | mean-solution start {it(meanst).mean():.0f} it | "
          f"learned {it(warm).mean():.0f} it ({t_warm:.3f}s), "
          f"kept {sum(r['used_warm_start'] for r in warm)}/{te.size}", flush=True)
    assert all(r["status"] == 0 and r["rel_kkt"] <= 1e-6 for r in warm + cold + meanst + wonly)
    # the network predicts the held-out solutions better than their training mean does
    assert err_l < 0.8 * err_m
    # against the method without it (cold start): the predicted point and weight cut the
    # iterations; the predicted weight alone does most of it
    assert it(warm).mean() < 0.8 * it(cold).mean()
    assert it(wonly).mean() < 0.8 * it(cold).mean()
    # Measured comparison with a constant prior (training-mean solution, geometric-mean
    # weight): on this family learned 780 vs mean 774 iterations, on the 5000-asset
    # family 3447 vs 3474; the last digits of a linearly converging method dominate, and a
    # better start shortens only the first phase.  Asserted: equal within 5 %.
    assert abs(it(warm).mean() - it(meanst).mean()) <= 0.05 * it(meanst).mean()
