"""Forward-mode dual numbers over NumPy arrays (oracle; test infrastructure).

A ``Dual`` carries a value array ``v`` and a derivative array ``d`` whose
last axis indexes seed directions.  All derivatives of the element residual
in the oracle come from here, never from a hand derivation, so they serve as
an independent check of the GPU's Jacobians (the exact derivatives of the
element residual, Appendix A, eq. (hdm_elem_jac1)).

Kink conventions: d|x| uses sign(0) = +1; maximum(a, b) follows ``a`` on a tie.
"""
from __future__ import annotations

import numpy as np


class Dual:
    __array_priority__ = 1000

    def __init__(self, v, d):
        self.v = np.asarray(v, dtype=np.float64)
        self.d = np.asarray(d, dtype=np.float64)

    # ----------------------------------------------------------- construction
    @staticmethod
    def const(v, nd: int) -> "Dual":
        v = np.asarray(v, dtype=np.float64)
        return Dual(v, np.zeros(v.shape + (nd,)))

    @staticmethod
    def seed(v, offset: int, nd: int) -> "Dual":
        """Independent variables: entry j (flattened over the trailing
        non-batch axes) gets direction offset + j.  The first axis is the
        batch axis and is not seeded separately."""
        v = np.asarray(v, dtype=np.float64)
        inner = int(np.prod(v.shape[1:]))
        d = np.zeros((v.shape[0], inner, nd))
        d[:, np.arange(inner), offset + np.arange(inner)] = 1.0
        return Dual(v, d.reshape(v.shape + (nd,)))

    @property
    def nd(self) -> int:
        return self.d.shape[-1]

    @property
    def shape(self):
        return self.v.shape

    def _wrap(self, o) -> "Dual":
        if isinstance(o, Dual):
            return o
        return Dual.const(o, self.nd)

    # ---------------------------------------------------------------- algebra
    def __add__(self, o):
        o = self._wrap(o)
        v = self.v + o.v
        return Dual(v, np.broadcast_to(self.d, v.shape + (self.nd,)) + o.d)

    __radd__ = __add__

    def __neg__(self):
        return Dual(-self.v, -self.d)

    def __sub__(self, o):
        return self + (-self._wrap(o))

    def __rsub__(self, o):
        return self._wrap(o) - self

    def __mul__(self, o):
        if not isinstance(o, Dual):
            o = np.asarray(o, dtype=np.float64)
            return Dual(self.v * o, self.d * o[..., None])
        return Dual(self.v * o.v, self.d * o.v[..., None] + self.v[..., None] * o.d)

    __rmul__ = __mul__

    def __truediv__(self, o):
        if not isinstance(o, Dual):
            o = np.asarray(o, dtype=np.float64)
            return Dual(self.v / o, self.d / o[..., None])
        q = self.v / o.v
        return Dual(q, (self.d - q[..., None] * o.d) / o.v[..., None])

    def __rtruediv__(self, o):
        return self._wrap(o) / self

    def __pow__(self, k):
        return Dual(self.v ** k, (k * self.v ** (k - 1))[..., None] * self.d)

    def __getitem__(self, key):
        v = self.v[key]
        if isinstance(key, tuple) and any(k is Ellipsis for k in key):
            d = self.d[key + (slice(None),)]
        elif key is Ellipsis:
            d = self.d
        else:
            d = self.d[key]
        return Dual(v, d)

    def sum(self, axis):
        ax = axis if axis >= 0 else axis - 1
        return Dual(self.v.sum(axis=axis), self.d.sum(axis=ax))


def lift(a, nd: int) -> Dual:
    return a if isinstance(a, Dual) else Dual.const(a, nd)


def _as_dual(a) -> Dual:
    return a if isinstance(a, Dual) else Dual.const(a, 0)


def sqrt(a: Dual) -> Dual:
    a = _as_dual(a)
    r = np.sqrt(a.v)
    return Dual(r, a.d / (2.0 * r)[..., None])


def exp(a: Dual) -> Dual:
    a = _as_dual(a)
    r = np.exp(a.v)
    return Dual(r, a.d * r[..., None])


def absd(a: Dual) -> Dual:
    a = _as_dual(a)
    s = np.where(a.v >= 0.0, 1.0, -1.0)
    return Dual(np.abs(a.v), a.d * s[..., None])


def where(cond, a: Dual, b: Dual) -> Dual:
    nd = max(x.nd for x in (a, b) if isinstance(x, Dual)) if any(isinstance(x, Dual) for x in (a, b)) else 0
    a, b = lift(a, nd), lift(b, nd)
    cond = np.asarray(cond)
    v = np.where(cond, a.v, b.v)
    d = np.where(cond[..., None], a.d, b.d)
    return Dual(v, d)


def maximum(a: Dual, b: Dual) -> Dual:
    a, b = _as_dual(a), _as_dual(b)
    return where(a.v >= b.v, a, b)


def stack(items, axis: int = -1) -> Dual:
    nd = next((x.nd for x in items if isinstance(x, Dual)), 0)
    items = [lift(x, nd) for x in items]
    shape = np.broadcast_shapes(*[x.v.shape for x in items])
    vs = [np.broadcast_to(x.v, shape) for x in items]
    ds = [np.broadcast_to(x.d, shape + (nd,)) for x in items]
    dax = axis if axis >= 0 else axis - 1
    return Dual(np.stack(vs, axis=axis), np.stack(ds, axis=dax))


def ein(spec: str, a, b) -> Dual:
    """einsum of two operands, either of which may be a Dual."""
    ins, out = spec.split("->")
    sa, sb = ins.split(",")
    da, db = isinstance(a, Dual), isinstance(b, Dual)
    av = a.v if da else np.asarray(a)
    bv = b.v if db else np.asarray(b)
    v = np.einsum(spec, av, bv)
    nd = a.nd if da else b.nd
    d = np.zeros(v.shape + (nd,))
    if da:
        d = d + np.einsum(f"{sa}Z,{sb}->{out}Z", a.d, bv)
    if db:
        d = d + np.einsum(f"{sa},{sb}Z->{out}Z", av, b.d)
    return Dual(v, d)
