"""Array back-ends for the oracle: numpy (float64 or long double) and torch (float64).

The oracle's physics is written once against this small interface so that the same
plain code gives double-precision results (numpy float64), a higher-precision ground
truth (numpy long double, 64-bit mantissa) and gradients (torch float64 autograd).
"""
from __future__ import annotations

import numpy as np


class NumpyOps:
    def __init__(self, dtype=np.float64):
        self.dtype = np.dtype(dtype)
        self.cdtype = np.complex128 if self.dtype == np.float64 else np.clongdouble
        self.pi = self.dtype.type(np.pi) if self.dtype == np.float64 else np.longdouble("3.14159265358979323846264338327950288")

    def asarray(self, x):
        return np.asarray(x, dtype=self.dtype)

    def const(self, v):
        return self.dtype.type(v)

    def zeros(self, shape, complex_=False):
        return np.zeros(shape, dtype=self.cdtype if complex_ else self.dtype)

    def cplx(self, re, im):
        return re.astype(self.cdtype) + 1j * im.astype(self.cdtype)

    def stack(self, xs, axis=-1):
        return np.stack(xs, axis=axis)

    def gather_legs(self, x, order):
        """x [B, n, ...] gathered along axis 1 by order [B, n]."""
        idx = order.astype(np.int64)
        idx = idx.reshape(idx.shape + (1,) * (x.ndim - 2))
        return np.take_along_axis(x, idx, axis=1)

    sqrt = staticmethod(np.sqrt)
    log = staticmethod(np.log)
    exp = staticmethod(np.exp)
    sin = staticmethod(np.sin)
    cos = staticmethod(np.cos)
    atan2 = staticmethod(np.arctan2)
    asinh = staticmethod(np.arcsinh)
    abs = staticmethod(np.abs)
    where = staticmethod(np.where)
    minimum = staticmethod(np.minimum)
    real = staticmethod(np.real)
    imag = staticmethod(np.imag)


class TorchOps:
    def __init__(self):
        import torch
        self.t = torch
        self.dtype = torch.float64
        self.cdtype = torch.complex128
        self.pi = float(np.pi)

    def asarray(self, x):
        if isinstance(x, self.t.Tensor):
            return x.to(self.dtype)
        return self.t.as_tensor(np.asarray(x, dtype=np.float64))

    def const(self, v):
        return float(v)

    def zeros(self, shape, complex_=False):
        return self.t.zeros(shape, dtype=self.cdtype if complex_ else self.dtype)

    def cplx(self, re, im):
        return self.t.complex(re, im)

    def stack(self, xs, axis=-1):
        return self.t.stack(xs, dim=axis)

    def gather_legs(self, x, order):
        idx = self.t.as_tensor(np.asarray(order, dtype=np.int64))
        idx = idx.reshape(tuple(idx.shape) + (1,) * (x.ndim - 2)).expand(x.shape)
        return self.t.gather(x, 1, idx)

    def sqrt(self, x):
        if not isinstance(x, self.t.Tensor):
            return float(np.sqrt(x))
        return self.t.sqrt(x)

    def log(self, x):
        return self.t.log(x)

    def exp(self, x):
        return self.t.exp(x)

    def sin(self, x):
        return self.t.sin(x)

    def cos(self, x):
        return self.t.cos(x)

    def atan2(self, y, x):
        return self.t.atan2(y, x)

    def asinh(self, x):
        return self.t.asinh(x)

    def abs(self, x):
        return self.t.abs(x)

    def where(self, c, a, b):
        return self.t.where(self.t.as_tensor(c), a, b)

    def minimum(self, a, b):
        return self.t.minimum(a, b)

    def real(self, x):
        return self.t.real(x)

    def imag(self, x):
        return self.t.imag(x)


NP64 = NumpyOps(np.float64)
NPLD = NumpyOps(np.longdouble)
