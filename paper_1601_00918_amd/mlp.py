"""Binding of the surrogate network's C ABI (include/lbm_mlp.h).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch provides device memory and streams.  The network, its parameter
layout and the loss are defined in include/lbm_mlp.h.
"""
import ctypes

from . import _lib
from ._lib import check

N_IN = 6
N_PARAMS = 34049


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    return ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)


def workspace_bytes(max_batch):
    return int(_lib.load().lbm_mlp_workspace_bytes(int(max_batch)))


def forward(params, X, y, ws, stream=None):
    """y[B] = net(params, X[B, 6]); all float32 CUDA tensors, contiguous."""
    B = X.shape[0]
    assert params.numel() == N_PARAMS and X.shape[1] == N_IN and y.numel() >= B
    check(_lib.load().lbm_mlp_forward(_ptr(params), _ptr(X), B, _ptr(y), _ptr(ws),
                                      ws.numel() * ws.element_size(), _stream(stream)),
          "lbm_mlp_forward")


def backward(params, X, y, t, grad, ws, loss=None, stream=None):
    """grad = dL/dparams of L = mean (y - t)^2 after forward() on the same ws."""
    B = X.shape[0]
    check(_lib.load().lbm_mlp_backward(_ptr(params), _ptr(X), _ptr(y), _ptr(t), B, _ptr(grad),
                                       _ptr(loss) if loss is not None else ctypes.c_void_p(0),
                                       _ptr(ws), ws.numel() * ws.element_size(),
                                       _stream(stream)),
          "lbm_mlp_backward")


NOALLOC_MAX_BATCH = 2048


def gradient_noalloc(params, X, t, y, grad, loss=None, stream=None):
    """forward() then backward() on one batch (B <= NOALLOC_MAX_BATCH) with
    the library's fixed device scratch instead of a workspace: nothing is
    allocated.  Calls that overlap on one device race."""
    B = X.shape[0]
    assert params.numel() == N_PARAMS and X.shape[1] == N_IN and y.numel() >= B
    check(_lib.load().lbm_mlp_gradient_noalloc(_ptr(params), _ptr(X), _ptr(t), B, _ptr(y),
                                               _ptr(grad),
                                               _ptr(loss) if loss is not None else ctypes.c_void_p(0),
                                               _stream(stream)),
          "lbm_mlp_gradient_noalloc")


def adam(params, grad, m, v, k, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    check(_lib.load().lbm_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(k),
                                   float(lr), float(beta1), float(beta2), float(eps),
                                   _stream(stream)),
          "lbm_mlp_adam")


class Network:
    """Parameters, Adam moments and workspace of one network on a device."""

    def __init__(self, params, max_batch, device="cuda"):
        import torch
        self.torch = torch
        self.params = torch.as_tensor(params, dtype=torch.float32).to(device).contiguous()
        assert self.params.numel() == N_PARAMS
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.k = 0
        self.max_batch = int(max_batch)
        self.ws = torch.empty(workspace_bytes(self.max_batch), dtype=torch.uint8, device=device)
        self.y = torch.empty(self.max_batch, dtype=torch.float32, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)

    def predict(self, X):
        """Network outputs for X [B, 6] (any B; chunks of max_batch)."""
        torch = self.torch
        X = torch.as_tensor(X, dtype=torch.float32).to(self.params.device).contiguous()
        out = torch.empty(X.shape[0], dtype=torch.float32, device=self.params.device)
        for s in range(0, X.shape[0], self.max_batch):
            xb = X[s:s + self.max_batch].contiguous()
            forward(self.params, xb, self.y, self.ws)
            out[s:s + xb.shape[0]] = self.y[:xb.shape[0]]
        return out

    def gradient(self, X, t):
        """(loss, grad) of the mean squared error on one batch (B <= max_batch)."""
        forward(self.params, X, self.y, self.ws)
        backward(self.params, X, self.y, t, self.grad, self.ws, self.loss)
        return self.loss, self.grad

    def train_step(self, X, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam step on the batch (X, t) (float32 CUDA tensors); returns
        the batch loss before the step (a device tensor)."""
        self.gradient(X, t)
        self.k += 1
        adam(self.params, self.grad, self.m, self.v, self.k, lr, beta1, beta2, eps)
        return self.loss
