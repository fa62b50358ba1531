"""The oracle's threaded timing mode (orc_set_threads) is bitwise the one-thread
oracle: every output element is computed by one thread with the sequential
operations in the sequential order, and every reduction stays sequential."""
import numpy as np
import pytest

import qpgen


@pytest.mark.parametrize("threads", [2, 8])
def test_threaded_solve_is_bitwise_sequential(orc, threads):
    cases = [(qpgen.tiny_random_qp(3), dict(eps=1e-7)),
             (qpgen.large_random_qp(seed=4, n=3000, m=1500), dict(eps=0.0, max_iter=320)),
             (qpgen.lasso_qp(seed=8, n_features=60, m_samples=300), dict(eps=1e-6)),
             (qpgen.tiny_random_qp(5), dict(eps=1e-6, restart_mode=orc.RESTART_HALVING))]
    for qp, kw in cases:
        s = orc.OracleSettings(**kw)
        orc.set_threads(1)
        try:
            ref = orc.solve(qp, s, log_cap=10000)
            orc.set_threads(threads)
            assert orc.get_threads() == threads
            got = orc.solve(qp, s, log_cap=10000)
        finally:
            orc.set_threads(1)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        for key in ("status", "iterations", "restarts", "rel_kkt", "primal_obj", "omega"):
            assert got[2][key] == ref[2][key], key
        assert got[3] == ref[3]
