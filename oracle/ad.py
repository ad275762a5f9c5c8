"""Forward-mode dual numbers over numpy arrays (the oracle's gradient tool).

A Dual carries a value array v and tangents d with shape (n_tangent,) + v.shape.
Arithmetic and the elementary functions below propagate first derivatives by
the chain rule; with the 13 parameters as seeds this yields d lnL / d theta
through exactly the code that computes lnL.  Works for real and complex values
(all functions used on complex values are holomorphic, except conj/real/imag
which act on value and tangents alike).
"""
import numpy as np


class Dual:
    __slots__ = ("v", "d")
    __array_priority__ = 1000
    __array_ufunc__ = None      # make numpy defer binary operators to Dual

    def __init__(self, v, d):
        self.v = np.asarray(v)
        d = np.asarray(d)
        shape = (d.shape[0],) + self.v.shape
        self.d = d if d.shape == shape else np.broadcast_to(d, shape)

    # -- helpers ---------------------------------------------------------------
    @property
    def n(self):
        return self.d.shape[0]

    def _expand(self, ndim):
        """Value and tangents with leading singleton axes up to ndim value dims."""
        k = ndim - self.v.ndim
        if k <= 0:
            return self.v, self.d
        v = self.v.reshape((1,) * k + self.v.shape)
        d = self.d.reshape((self.d.shape[0],) + (1,) * k + self.v.shape)
        return v, d

    # -- arithmetic ------------------------------------------------------------
    def __add__(self, o):
        if isinstance(o, Dual):
            nd = max(self.v.ndim, o.v.ndim)
            av, ad = self._expand(nd)
            bv, bd = o._expand(nd)
            return Dual(av + bv, ad + bd)
        o = np.asarray(o)
        nd = max(self.v.ndim, o.ndim)
        av, ad = self._expand(nd)
        return Dual(av + o, ad)

    __radd__ = __add__

    def __neg__(self):
        return Dual(-self.v, -self.d)

    def __sub__(self, o):
        return self + (-o if isinstance(o, Dual) else -np.asarray(o))

    def __rsub__(self, o):
        return (-self) + o

    def __mul__(self, o):
        if isinstance(o, Dual):
            nd = max(self.v.ndim, o.v.ndim)
            av, ad = self._expand(nd)
            bv, bd = o._expand(nd)
            return Dual(av * bv, ad * bv + av * bd)
        o = np.asarray(o)
        nd = max(self.v.ndim, o.ndim)
        av, ad = self._expand(nd)
        return Dual(av * o, ad * o)

    __rmul__ = __mul__

    def __truediv__(self, o):
        if isinstance(o, Dual):
            return self * o.reciprocal()
        return self * (1.0 / np.asarray(o))

    def __rtruediv__(self, o):
        return self.reciprocal() * o

    def reciprocal(self):
        r = 1.0 / self.v
        return Dual(r, -self.d * (r * r))

    def __pow__(self, p):
        if isinstance(p, Dual):
            return exp(log(self) * p)
        p = float(p)
        if p == 2.0:
            return self * self
        vp = self.v ** p
        return Dual(vp, self.d * (p * self.v ** (p - 1.0)))

    def __rpow__(self, base):
        return exp(self * np.log(base))

    # -- complex parts -----------------------------------------------------------
    @property
    def real(self):
        return Dual(np.real(self.v), np.real(self.d))

    @property
    def imag(self):
        return Dual(np.imag(self.v), np.imag(self.d))

    def conj(self):
        return Dual(np.conj(self.v), np.conj(self.d))

    # -- container-ish -------------------------------------------------------------
    def __getitem__(self, idx):
        if not isinstance(idx, tuple):
            idx = (idx,)
        return Dual(self.v[idx], self.d[(slice(None),) + idx])

    @property
    def shape(self):
        return self.v.shape

    def sum(self, axis=None):
        if axis is None:
            return Dual(self.v.sum(), self.d.reshape(self.d.shape[0], -1).sum(axis=1))
        ax = axis if axis >= 0 else self.v.ndim + axis
        return Dual(self.v.sum(axis=ax), self.d.sum(axis=ax + 1))

    def __repr__(self):
        return f"Dual(v={self.v!r}, d.shape={self.d.shape})"


def seed(values, idx=None, n=None):
    """Independent variables: a Dual for each entry of `values` (1-D), with a
    unit tangent in slot idx[i] (default i) of n tangents."""
    values = np.asarray(values, dtype=np.float64)
    n = values.shape[-1] if n is None else n
    out = []
    for i in range(values.shape[-1]):
        d = np.zeros((n,) + values.shape[:-1])
        d[i if idx is None else idx[i]] = 1.0
        out.append(Dual(values[..., i], d))
    return out


def value(x):
    return x.v if isinstance(x, Dual) else np.asarray(x)


def tangent(x, n):
    if isinstance(x, Dual):
        return x.d
    x = np.asarray(x)
    return np.zeros((n,) + x.shape, dtype=x.dtype)


def _unary(x, f, df):
    if isinstance(x, Dual):
        return Dual(f(x.v), x.d * df(x.v))
    return f(x)


def sin(x):
    return _unary(x, np.sin, np.cos)


def cos(x):
    return _unary(x, np.cos, lambda v: -np.sin(v))


def exp(x):
    if isinstance(x, Dual):
        e = np.exp(x.v)
        return Dual(e, x.d * e)
    return np.exp(x)


def log(x):
    return _unary(x, np.log, lambda v: 1.0 / v)


def sqrt(x):
    if isinstance(x, Dual):
        s = np.sqrt(x.v)
        return Dual(s, x.d * (0.5 / s))
    return np.sqrt(x)


def arctan(x):
    return _unary(x, np.arctan, lambda v: 1.0 / (1.0 + v * v))


def arccos(x):
    return _unary(x, np.arccos, lambda v: -1.0 / np.sqrt(1.0 - v * v))


def tanh(x):
    return _unary(x, np.tanh, lambda v: 1.0 - np.tanh(v) ** 2)


def cbrt(x):
    if isinstance(x, Dual):
        c = np.cbrt(x.v)
        return Dual(c, x.d * (1.0 / (3.0 * c * c)))
    return np.cbrt(x)


def where(cond, a, b):
    """Elementwise select that keeps tangents of the chosen branch."""
    if not isinstance(a, Dual) and not isinstance(b, Dual):
        return np.where(cond, a, b)
    n = a.n if isinstance(a, Dual) else b.n
    av, bv = value(a), value(b)
    ad, bd = tangent(a, n), tangent(b, n)
    return Dual(np.where(cond, av, bv), np.where(cond, ad, bd))
