"""Oracle of the scalar-expression evaluator -- TEST INFRASTRUCTURE ONLY.

The plain definition (Section 3.2.1: an expression over scalars, evaluated
to one value per output): a postfix program run on a stack of Python floats
(IEEE double), one operation at a time, in program order.  Op numbering is
the C ABI's (restated here, not imported: the oracle shares nothing with the
product package).
"""
from __future__ import annotations

import math

INPUT, CONST = 1, 2
NEG, RECIP, SQRT, ABS, EXP, LOG, SIN, COS = 10, 11, 12, 13, 14, 15, 16, 17
ADD, SUB, MUL, DIV, MIN, MAX = 20, 21, 22, 23, 24, 25
OUTPUT = 30


def _minnum(a, b):
    if math.isnan(a):
        return b
    if math.isnan(b):
        return a
    return a if a < b or (a == b and math.copysign(1.0, a) < 0) else b


def _maxnum(a, b):
    if math.isnan(a):
        return b
    if math.isnan(b):
        return a
    return a if a > b or (a == b and math.copysign(1.0, a) > 0) else b


def _div(a, b):
    if b == 0.0:
        if a == 0.0 or math.isnan(a):
            return math.nan
        return math.copysign(math.inf, a) * math.copysign(1.0, b)
    return a / b


def _sqrt(a):
    if math.isnan(a) or a < 0:
        return math.nan
    return math.sqrt(a)


def _exp(a):
    try:
        return math.exp(a)
    except OverflowError:
        return math.inf


UNARY = {NEG: lambda a: -a, RECIP: lambda a: _div(1.0, a), SQRT: _sqrt, ABS: abs,
         EXP: _exp, LOG: lambda a: math.log(a) if a > 0 else (-math.inf if a == 0 else math.nan),
         SIN: math.sin, COS: math.cos}
BINARY = {ADD: lambda a, b: a + b, SUB: lambda a, b: a - b, MUL: lambda a, b: a * b, DIV: _div,
          MIN: _minnum, MAX: _maxnum}


def eval_postfix(tokens, inputs, noutputs):
    """Runs the program on the inputs; returns the list of outputs."""
    stack, out = [], [None] * noutputs
    for op, arg, value in tokens:
        if op == INPUT:
            stack.append(float(inputs[arg]))
        elif op == CONST:
            stack.append(float(value))
        elif op in UNARY:
            stack.append(UNARY[op](stack.pop()))
        elif op in BINARY:
            b = stack.pop()
            a = stack.pop()
            stack.append(BINARY[op](a, b))
        elif op == OUTPUT:
            out[arg] = stack.pop()
        else:
            raise ValueError(f"unknown op {op}")
    if stack or any(o is None for o in out):
        raise ValueError("malformed program")
    return out
