"""Symbolic scalar expressions over device scalars (the expression-template
side of Section 3.2.1): Python operators on ``Sym`` build the postfix token
program that ``apcg_expr_compile`` (Eval) turns into one device kernel.

    x, y, z = Sym.inputs(3)
    e = Eval([(x + y) / z, sqrt(x * x + y * y)], ninputs=3)
    e.execute(ctx, [sx, sy, sz], [s_out0, s_out1])   # one launch, two results

Nothing here computes: the arithmetic runs on the device.
"""
from __future__ import annotations

from . import _capi
from . import apcg_expr_compile, apcg_expr_destroy, apcg_expr_execute, apcg_expr_stats


class Sym:
    """A symbolic expression: its postfix tokens (op, arg, value)."""

    def __init__(self, tokens):
        self.tokens = list(tokens)

    @staticmethod
    def input(i: int) -> "Sym":
        return Sym([(_capi.APCG_EXPR_INPUT, i, 0.0)])

    @staticmethod
    def inputs(n: int):
        return [Sym.input(i) for i in range(n)]

    def _bin(self, other, op, swap=False):
        o = other if isinstance(other, Sym) else const(other)
        a, b = (o, self) if swap else (self, o)
        return Sym(a.tokens + b.tokens + [(op, 0, 0.0)])

    def __add__(self, o):
        return self._bin(o, _capi.APCG_EXPR_ADD)

    def __radd__(self, o):
        return self._bin(o, _capi.APCG_EXPR_ADD, True)

    def __sub__(self, o):
        return self._bin(o, _capi.APCG_EXPR_SUB)

    def __rsub__(self, o):
        return self._bin(o, _capi.APCG_EXPR_SUB, True)

    def __mul__(self, o):
        return self._bin(o, _capi.APCG_EXPR_MUL)

    def __rmul__(self, o):
        return self._bin(o, _capi.APCG_EXPR_MUL, True)

    def __truediv__(self, o):
        return self._bin(o, _capi.APCG_EXPR_DIV)

    def __rtruediv__(self, o):
        return self._bin(o, _capi.APCG_EXPR_DIV, True)

    def __neg__(self):
        return _un(self, _capi.APCG_EXPR_NEG)


def const(v: float) -> Sym:
    return Sym([(_capi.APCG_EXPR_CONST, 0, float(v))])


def _un(x, op) -> Sym:
    x = x if isinstance(x, Sym) else const(x)
    return Sym(x.tokens + [(op, 0, 0.0)])


def recip(x):
    return _un(x, _capi.APCG_EXPR_RECIP)


def sqrt(x):
    return _un(x, _capi.APCG_EXPR_SQRT)


def fabs(x):
    return _un(x, _capi.APCG_EXPR_ABS)


def exp(x):
    return _un(x, _capi.APCG_EXPR_EXP)


def log(x):
    return _un(x, _capi.APCG_EXPR_LOG)


def sin(x):
    return _un(x, _capi.APCG_EXPR_SIN)


def cos(x):
    return _un(x, _capi.APCG_EXPR_COS)


def minimum(a, b):
    a = a if isinstance(a, Sym) else const(a)
    return a._bin(b, _capi.APCG_EXPR_MIN)


def maximum(a, b):
    a = a if isinstance(a, Sym) else const(a)
    return a._bin(b, _capi.APCG_EXPR_MAX)


def program(outputs) -> list:
    """Postfix tokens computing every expression of ``outputs`` in order."""
    toks = []
    for k, e in enumerate(outputs):
        e = e if isinstance(e, Sym) else const(e)
        toks += e.tokens + [(_capi.APCG_EXPR_OUTPUT, k, 0.0)]
    return toks


class Eval:
    """A compiled (executable) expression program: one or more outputs
    (MultiEval) over ``ninputs`` device scalars."""

    def __init__(self, outputs, ninputs: int):
        outputs = list(outputs)
        self.tokens = program(outputs)
        self.ninputs = ninputs
        self.noutputs = len(outputs)
        self.h = apcg_expr_compile(self.tokens, ninputs, self.noutputs)

    def stats(self) -> dict:
        return apcg_expr_stats(self.h)

    def execute(self, ctx, inputs, outputs) -> None:
        apcg_expr_execute(self.h, ctx, list(inputs), list(outputs))

    def close(self) -> None:
        if self.h is not None:
            apcg_expr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
