"""Python binding of the sampler's BF16 MLP (include/rad_mlp.h): marshalling only.

Training and inference run in librad's HIP kernels; torch holds the device
buffers and supplies the stream.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import rad

_bound = False


def _lib():
    global _bound
    L = rad.lib()
    if not _bound:
        P, I, I64, S, F = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t, ctypes.c_float
        FP = ctypes.POINTER(ctypes.c_float)
        sig = {
            "rad_mlp_create": (I, [I, I, ctypes.c_uint64, P, ctypes.POINTER(P)]),
            "rad_mlp_free": (None, [P]),
            "rad_mlp_param_count": (I64, [P]),
            "rad_mlp_get_params": (I, [P, FP, P]),
            "rad_mlp_set_params": (I, [P, FP, P]),
            "rad_mlp_get_adam": (I, [P, FP, FP, ctypes.POINTER(I64), P]),
            "rad_mlp_set_adam": (I, [P, FP, FP, I64, P]),
            "rad_mlp_workspace_bytes": (S, [P, I, I, I]),
            "rad_mlp_grad": (I, [P, P, I, P, P, P, I, P, P, P, S, P]),
            "rad_mlp_adam": (I, [P, P, F, F, F, F, P]),
            "rad_mlp_forward": (I, [P, P, I, P, P, I, P, P, S, P]),
            "rad_mlp_grid_workspace_bytes": (S, [P, I]),
            "rad_mlp_forward_grid": (I, [P, P, I, P, I64, P, P, S, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return L


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class MLP:
    """in = [n_feat trajectory features, n_point point inputs] -> 256 -> 256 -> 256 -> 1."""

    def __init__(self, n_feat, n_point=3, seed=0, stream=None):
        self.n_feat, self.n_point = int(n_feat), int(n_point)
        h = ctypes.c_void_p()
        rad._check(_lib().rad_mlp_create(self.n_feat, self.n_point, int(seed) & (2 ** 64 - 1),
                                         rad._stream(stream), ctypes.byref(h)), "rad_mlp_create")
        self.handle = h
        self._ws = None

    @property
    def param_count(self):
        return int(_lib().rad_mlp_param_count(self.handle))

    def get_params(self, stream=None):
        out = np.empty(self.param_count, dtype=np.float32)
        rad._check(_lib().rad_mlp_get_params(self.handle, _fp(out), rad._stream(stream)),
                   "rad_mlp_get_params")
        return out

    def set_params(self, theta, stream=None):
        t = _f32(theta)
        if t.size != self.param_count:
            raise ValueError("expected %d parameters" % self.param_count)
        rad._check(_lib().rad_mlp_set_params(self.handle, _fp(t), rad._stream(stream)),
                   "rad_mlp_set_params")

    def get_adam(self, stream=None):
        m1 = np.empty(self.param_count, dtype=np.float32)
        m2 = np.empty_like(m1)
        step = ctypes.c_int64()
        rad._check(_lib().rad_mlp_get_adam(self.handle, _fp(m1), _fp(m2), ctypes.byref(step),
                                           rad._stream(stream)), "rad_mlp_get_adam")
        return m1, m2, step.value

    def set_adam(self, m1, m2, step, stream=None):
        a, b = _f32(m1), _f32(m2)
        rad._check(_lib().rad_mlp_set_adam(self.handle, _fp(a), _fp(b), int(step),
                                           rad._stream(stream)), "rad_mlp_set_adam")

    def save(self, path):
        """Checkpoint: parameters, Adam moments and step (NumPy .npz, no pickles)."""
        m1, m2, step = self.get_adam()
        np.savez(path, params=self.get_params(), m1=m1, m2=m2, step=np.int64(step),
                 shape=np.array([self.n_feat, self.n_point], dtype=np.int64))

    def load(self, path):
        with np.load(path, allow_pickle=False) as z:
            if tuple(z["shape"]) != (self.n_feat, self.n_point):
                raise ValueError("checkpoint is for a different input shape")
            self.set_params(z["params"])
            self.set_adam(z["m1"], z["m2"], int(z["step"]))

    def _workspace(self, batch, n_traj, training=True):
        import torch
        nb = int(_lib().rad_mlp_workspace_bytes(self.handle, int(batch), int(n_traj), int(training)))
        if self._ws is None or self._ws.numel() < nb:
            self._ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        return self._ws

    @staticmethod
    def _check_inputs(feat, traj, x, n_point):
        import torch
        for t, dt in ((feat, torch.float32), (traj, torch.int32), (x, torch.float32)):
            if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
                raise ValueError("feat/x must be contiguous float32 and traj int32 CUDA tensors")
        if x.dim() != 2 or x.shape[1] != n_point or traj.numel() != x.shape[0]:
            raise ValueError("x must be [batch, n_point] and traj [batch]")

    def grad(self, feat, traj, x, target, grad=None, loss_sum=None, stream=None):
        """Gradient of the mean squared error; returns (grad [P], loss_sum [1]) tensors."""
        import torch
        self._check_inputs(feat, traj, x, self.n_point)
        B = x.shape[0]
        if grad is None:
            grad = torch.empty(self.param_count, dtype=torch.float32, device="cuda")
        if loss_sum is None:
            loss_sum = torch.empty(1, dtype=torch.float32, device="cuda")
        ws = self._workspace(B, feat.shape[0])
        rad._check(_lib().rad_mlp_grad(self.handle, rad._dptr(feat), feat.shape[0], rad._dptr(traj),
                                       rad._dptr(x), rad._dptr(target), B, rad._dptr(grad),
                                       rad._dptr(loss_sum), rad._dptr(ws), ws.numel(),
                                       rad._stream(stream)), "rad_mlp_grad")
        return grad, loss_sum

    def adam(self, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        rad._check(_lib().rad_mlp_adam(self.handle, rad._dptr(grad), float(lr), float(beta1),
                                       float(beta2), float(eps), rad._stream(stream)), "rad_mlp_adam")

    def train_step(self, feat, traj, x, target, lr, **adam_kw):
        """grad + Adam; returns the batch's summed squared error (a device tensor [1]; the
        mean is that over the batch size)."""
        g, ls = self.grad(feat, traj, x, target)
        self.adam(g, lr, **adam_kw)
        return ls

    def forward(self, feat, traj, x, y=None, stream=None):
        """Inference (trajectory features folded into a per-trajectory bias)."""
        import torch
        self._check_inputs(feat, traj, x, self.n_point)
        B = x.shape[0]
        if y is None:
            y = torch.empty(B, dtype=torch.float32, device="cuda")
        ws = self._workspace(B, feat.shape[0], training=False)
        rad._check(_lib().rad_mlp_forward(self.handle, rad._dptr(feat), feat.shape[0], rad._dptr(traj),
                                          rad._dptr(x), B, rad._dptr(y), rad._dptr(ws), ws.numel(),
                                          rad._stream(stream)), "rad_mlp_forward")
        return y

    def forward_grid(self, feat, x, y=None, stream=None):
        """Inference at every (trajectory, point) pair: feat [n_traj, n_feat], x the point
        table [n_pts, n_point]; returns y [n_traj, n_pts] (fused kernel, n_point <= 8)."""
        import torch
        for t in (feat, x):
            if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
                raise ValueError("feat and x must be contiguous float32 CUDA tensors")
        if x.dim() != 2 or x.shape[1] != self.n_point or feat.dim() != 2:
            raise ValueError("x must be [n_pts, n_point] and feat [n_traj, n_feat]")
        n_traj, n_pts = feat.shape[0], x.shape[0]
        if y is None:
            y = torch.empty((n_traj, n_pts), dtype=torch.float32, device="cuda")
        if tuple(y.shape) != (n_traj, n_pts) or not y.is_contiguous() or y.dtype != torch.float32:
            raise ValueError("y must be a contiguous float32 [n_traj, n_pts] tensor")
        nb = int(_lib().rad_mlp_grid_workspace_bytes(self.handle, int(n_traj)))
        if self._ws is None or self._ws.numel() < nb:
            self._ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
        rad._check(_lib().rad_mlp_forward_grid(self.handle, rad._dptr(feat), int(n_traj), rad._dptr(x), int(n_pts),
                                               rad._dptr(y), rad._dptr(self._ws), self._ws.numel(),
                                               rad._stream(stream)), "rad_mlp_forward_grid")
        return y

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            _lib().rad_mlp_free(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
