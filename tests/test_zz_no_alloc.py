"""qp_mlp_forward_noalloc (workspace in the library's static device memory) against
qp_mlp_forward on the same handle: the same kernels on the same operands, so the
outputs agree bit for bit; two calls in a row, the second with a smaller batch, so
a stale workspace (the K padding of a layer's input) would show."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    return torch


def _mlp(sizes, batch, seed):
    from paper_2311_07710_amd.mlp import MLP, init_params
    m = MLP(sizes, max_batch=batch)
    m.set_params(init_params(sizes, seed=seed, out_scale=1.0))
    return m


@pytest.mark.parametrize("sizes,batches", [
    ([37, 64, 48, 29], (50, 7)),          # padded layer widths (37, 48 and 29 are not multiples of 32)
    ([10001, 512, 512, 5202], (256, 33)),  # the warm-start network, split-K on every product
])
def test_noalloc_forward_matches_forward(torch_cuda, sizes, batches):
    torch = torch_cuda
    rng = np.random.default_rng(11)
    m = _mlp(sizes, batches[0], seed=3)
    try:
        for batch in batches:
            print(f"noalloc forward: sizes={sizes} batch={batch}", flush=True)
            X = torch.from_numpy(rng.standard_normal((batch, sizes[0])).astype(np.float32)).cuda()
            # a different input first, so the workspace holds other values than this call's
            m.forward_noalloc(torch.from_numpy(
                rng.standard_normal((batches[0], sizes[0])).astype(np.float32)).cuda())
            got = m.forward_noalloc(X).cpu().numpy()
            want = m.forward(X).cpu().numpy()
            assert got.shape == want.shape == (batch, sizes[-1])
            assert np.array_equal(got, want), float(np.max(np.abs(got - want)))
    finally:
        m.close()


def test_noalloc_rejects_workspace_beyond_limit(torch_cuda):
    """A batch whose activations and partials exceed the fixed workspace is refused before
    any device work, with the limit in the message; the handle stays usable."""
    torch = torch_cuda
    from paper_2311_07710_amd import _binding as B
    lib = B.load()
    sizes, big = [20000, 64, 8], 1024   # 2 x 1024 x 20000 BF16 alone is 78 MiB
    m = _mlp(sizes, big, seed=4)
    try:
        X = torch.zeros(big, sizes[0], dtype=torch.float32, device="cuda")
        out = torch.empty(big, sizes[-1], dtype=torch.float32, device="cuda")
        rc = lib.qp_mlp_forward_noalloc(m.h, X.data_ptr(), big, out.data_ptr())
        assert rc == B.QP_ERR_INVALID_ARGUMENT
        msg = lib.qp_last_error().decode()
        assert "limit" in msg, msg
        small = X[:16].contiguous()
        got = m.forward_noalloc(small).cpu().numpy()
        want = m.forward(small).cpu().numpy()
        assert np.array_equal(got, want)
    finally:
        m.close()
