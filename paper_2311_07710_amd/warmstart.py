"""Learned warm start for a parametrised portfolio-QP family.

Every instance of the family shares D and F and differs in mu (the return
vector) and the budget.  The MLP maps [mu, (mu - mu_bar)/sigma, budget] to the
primal point (x, y_factors), the duals of all rows and log(omega) of a cold
rAPDHG solve; it is trained on solutions the batched solver produced.  A
prediction is only a starting point: qp_batch_solve with warm_fallback = 1
keeps it only if its relative KKT error beats the cold start's, and the
solve's own termination test checks the result.

Host code here only prepares arrays (standardisation) and drives the library;
the solves, the forward/backward passes and the Adam steps run on the GPU.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from .mlp import MLP, init_params
from .solver import BatchSolver, Settings


def features(fam, idx) -> np.ndarray:
    idx = np.asarray(idx)
    mu = fam.mu[idx]
    std = (mu - fam.mu_bar[None, :]) / fam.mu_sigma
    return np.hstack([mu, std, fam.budget[idx][:, None]]).astype(np.float64)


def targets(x, y, omega) -> np.ndarray:
    return np.hstack([x, y, np.log(np.asarray(omega))[:, None]])


def family_norms(fam, settings: Settings | None = None):
    """||A||_2 and ||Q||_2 of the family.  A and Q are the same for every member
    (only c and b vary), so one power iteration on member 0 serves them all."""
    from .solver import Solver
    with Solver(fam.instance(0), settings or Settings()) as s:
        return s.norms()


def solve_family(fam, idx, settings: Settings, x0=None, y0=None, omega0=None, threads=None,
                 chunk: int = 0, log=None):
    """Batched solves of family members idx; returns (X [k,n], Y [k,m], results, seconds).

    With chunk > 0 the members are solved in launches of at most chunk instances
    (log receives one line per launch).  Unless settings carries norm overrides,
    the family's norms are computed once and passed to every launch."""
    import dataclasses
    idx = np.asarray(idx)
    if settings.norm_A <= 0.0 or settings.norm_Q <= 0.0:
        nA, nQ = family_norms(fam, settings)
        settings = dataclasses.replace(settings, norm_A=nA, norm_Q=nQ)
    n, m = fam.base.n, fam.base.m
    k = len(idx)
    step = k if chunk <= 0 else chunk
    X, Y, res, dt = np.zeros((k, n)), np.zeros((k, m)), [], 0.0
    for s0 in range(0, k, step):
        sl = slice(s0, min(k, s0 + step))
        bs = BatchSolver(fam.batch(idx[sl]), settings)
        if threads is not None:
            bs.set_threads(threads)
        t = time.perf_counter()
        x, y, r = bs.solve(x0=None if x0 is None else np.ascontiguousarray(x0[sl]).ravel(),
                           y0=None if y0 is None else np.ascontiguousarray(y0[sl]).ravel(),
                           omega0=None if omega0 is None else np.asarray(omega0)[sl])
        dt += time.perf_counter() - t
        bs.close()
        cnt = sl.stop - sl.start
        X[sl] = x.reshape(cnt, n)
        Y[sl] = y.reshape(cnt, m)
        res.extend(r)
        if log:
            its = sum(q["iterations"] for q in r)
            log(f"solved {sl.stop}/{k} (chunk {cnt}, {its} iterations, {dt:.2f} s total)")
    return X, Y, res, dt


@dataclass
class WarmStartModel:
    mlp: MLP
    f_mean: np.ndarray
    f_std: np.ndarray
    t_mean: np.ndarray
    t_std: np.ndarray
    n: int
    m: int
    history: list

    def predict(self, F: np.ndarray, batch: int = 0):
        import torch
        batch = self.mlp.max_batch if batch <= 0 else min(batch, self.mlp.max_batch)
        Z = ((F - self.f_mean) / self.f_std).astype(np.float32)
        outs = []
        for s in range(0, Z.shape[0], batch):
            xb = torch.from_numpy(Z[s:s + batch]).cuda().contiguous()
            outs.append(self.mlp.forward(xb).cpu().numpy().astype(np.float64))
        P = np.vstack(outs) * self.t_std + self.t_mean
        n, m = self.n, self.m
        return P[:, :n], P[:, n:n + m], np.exp(P[:, n + m])


def train(F: np.ndarray, T: np.ndarray, n: int, m: int, hidden=(512, 512), epochs: int = 40,
          batch: int = 256, lr: float = 1e-3, seed: int = 0, log=None) -> WarmStartModel:
    import torch
    f_mean, f_std = F.mean(axis=0), F.std(axis=0)
    f_std = np.where(f_std > 1e-8, f_std, 1.0)
    t_mean, t_std = T.mean(axis=0), T.std(axis=0)
    t_std = np.where(t_std > 1e-8, t_std, 1.0)
    Zf = torch.from_numpy(((F - f_mean) / f_std).astype(np.float32)).cuda()
    Zt = torch.from_numpy(((T - t_mean) / t_std).astype(np.float32)).cuda()
    sizes = [F.shape[1], *hidden, T.shape[1]]
    mlp = MLP(sizes, max_batch=batch)
    mlp.set_params(init_params(sizes, seed=seed))
    rng = np.random.default_rng(seed + 1)
    step = 0
    hist = []
    N = F.shape[0]
    for ep in range(epochs):
        # the minibatch rows are gathered by the library's kernels (no device copy here)
        perm = torch.from_numpy(rng.permutation(N).astype(np.int32)).cuda()
        tot, cnt = 0.0, 0
        for s in range(0, N - batch + 1, batch):
            sel = perm[s:s + batch]
            mlp.forward_rows(Zf, sel)
            loss = mlp.backward_rows(Zt, sel)
            step += 1
            mlp.adam_step(lr=lr, step=step)
            tot += loss
            cnt += 1
        hist.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep + 1}/{epochs} loss {hist[-1]:.5f}")
    return WarmStartModel(mlp, f_mean, f_std, t_mean, t_std, n, m, hist)
