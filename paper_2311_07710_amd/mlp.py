"""Python handle of the BF16/FP32 warm-start MLP (include/qp_mlp.h).

Marshalling only: forward, backward and Adam run in the library's MFMA
kernels.  Inputs and targets are torch CUDA float32 tensors (device memory).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _binding as B


class MLP:
    def __init__(self, sizes, max_batch: int, device: int = 0):
        self.lib = B.load()
        self.sizes = [int(s) for s in sizes]
        self.max_batch = int(max_batch)
        arr = np.asarray(self.sizes, dtype=np.int32)
        h = C.c_void_p()
        B.check(self.lib.qp_mlp_create(len(self.sizes) - 1, arr.ctypes.data, self.max_batch,
                                       int(device), C.byref(h)))
        self.h = h
        self.n_params = int(self.lib.qp_mlp_num_params(self.h))

    def close(self):
        if getattr(self, "h", None):
            self.lib.qp_mlp_free(self.h)
            self.h = None

    __del__ = close

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == self.n_params
        B.check(self.lib.qp_mlp_set_params(self.h, p.ctypes.data))

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.n_params, dtype=np.float32)
        B.check(self.lib.qp_mlp_get_params(self.h, p.ctypes.data))
        return p

    def get_grads(self) -> np.ndarray:
        g = np.zeros(self.n_params, dtype=np.float32)
        B.check(self.lib.qp_mlp_get_grads(self.h, g.ctypes.data))
        return g

    def set_grads(self, grads):
        g = np.ascontiguousarray(grads, dtype=np.float32)
        assert g.size == self.n_params
        B.check(self.lib.qp_mlp_set_grads(self.h, g.ctypes.data))

    def forward_rows(self, x_all, rows):
        """Forward on the minibatch x_all[rows] (rows: CUDA int32 tensor), gathered by the
        library's input conversion kernel."""
        import torch
        assert x_all.is_cuda and x_all.dtype == torch.float32 and x_all.is_contiguous()
        assert rows.is_cuda and rows.dtype == torch.int32 and rows.is_contiguous()
        out = torch.empty(rows.shape[0], self.sizes[-1], dtype=torch.float32, device=x_all.device)
        torch.cuda.current_stream().synchronize()
        B.check(self.lib.qp_mlp_forward_rows(self.h, x_all.data_ptr(), x_all.shape[0],
                                             rows.data_ptr(), rows.shape[0], out.data_ptr()))
        return out

    def backward_rows(self, t_all, rows) -> float:
        import torch
        assert t_all.is_cuda and t_all.dtype == torch.float32 and t_all.is_contiguous()
        assert rows.is_cuda and rows.dtype == torch.int32 and rows.is_contiguous()
        torch.cuda.current_stream().synchronize()
        loss = C.c_float()
        B.check(self.lib.qp_mlp_backward_rows(self.h, t_all.data_ptr(), t_all.shape[0],
                                              rows.data_ptr(), rows.shape[0], C.byref(loss)))
        return float(loss.value)

    def forward(self, x):
        import torch
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()
        out = torch.empty(x.shape[0], self.sizes[-1], dtype=torch.float32, device=x.device)
        torch.cuda.current_stream().synchronize()
        B.check(self.lib.qp_mlp_forward(self.h, x.data_ptr(), x.shape[0], out.data_ptr()))
        return out

    def forward_noalloc(self, x, out=None):
        """Inference through qp_mlp_forward_noalloc (workspace in the library's static
        device memory; no activations kept for backward)."""
        import torch
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()
        if out is None:
            out = torch.empty(x.shape[0], self.sizes[-1], dtype=torch.float32, device=x.device)
        assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
        torch.cuda.current_stream().synchronize()
        B.check(self.lib.qp_mlp_forward_noalloc(self.h, x.data_ptr(), x.shape[0], out.data_ptr()))
        return out

    def backward(self, target) -> float:
        import torch
        assert target.is_cuda and target.dtype == torch.float32 and target.is_contiguous()
        torch.cuda.current_stream().synchronize()
        loss = C.c_float()
        B.check(self.lib.qp_mlp_backward(self.h, target.data_ptr(), target.shape[0], C.byref(loss)))
        return float(loss.value)

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, step=1):
        B.check(self.lib.qp_mlp_adam_step(self.h, float(lr), float(beta1), float(beta2),
                                          float(eps), int(step)))


def init_params(sizes, seed: int = 0, out_scale: float = 0.1) -> np.ndarray:
    """He-uniform weights, zero biases; the output layer scaled by out_scale."""
    rng = np.random.default_rng(seed)
    parts = []
    L = len(sizes) - 1
    for l in range(L):
        fan_in = sizes[l]
        a = np.sqrt(6.0 / fan_in) * (out_scale if l == L - 1 else 1.0)
        parts.append(rng.uniform(-a, a, sizes[l + 1] * sizes[l]))
        parts.append(np.zeros(sizes[l + 1]))
    return np.concatenate(parts).astype(np.float32)
