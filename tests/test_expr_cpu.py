"""Scalar expressions (Section 3.2.1), CPU side: the oracle's evaluator
against closed forms, and the compiler (Eval: validation, common
subexpressions, constant folding, exact rewrites), which runs on the host
and needs no GPU.  Execution on the device is tested in test_gpu_model.py."""
import math

import pytest

from oracle import expr as OX


def tok(*t):
    return list(t)


def test_oracle_postfix_closed_forms():
    # (x + y) * z - x / y with x = 3, y = 4, z = 5: 35 - 0.75
    prog = [(OX.INPUT, 0, 0), (OX.INPUT, 1, 0), (OX.ADD, 0, 0), (OX.INPUT, 2, 0), (OX.MUL, 0, 0),
            (OX.INPUT, 0, 0), (OX.INPUT, 1, 0), (OX.DIV, 0, 0), (OX.SUB, 0, 0), (OX.OUTPUT, 0, 0)]
    assert OX.eval_postfix(prog, [3.0, 4.0, 5.0], 1) == [34.25]
    # several outputs; sqrt of a perfect square; recip of a power of two
    prog = [(OX.CONST, 0, 144.0), (OX.SQRT, 0, 0), (OX.OUTPUT, 1, 0), (OX.CONST, 0, 8.0), (OX.RECIP, 0, 0),
            (OX.OUTPUT, 0, 0)]
    assert OX.eval_postfix(prog, [], 2) == [0.125, 12.0]
    # minNum / maxNum: a NaN operand yields the other
    nan = math.nan
    assert OX.eval_postfix([(OX.CONST, 0, nan), (OX.CONST, 0, 2.0), (OX.MIN, 0, 0), (OX.OUTPUT, 0, 0)], [], 1) == [2.0]
    assert OX.eval_postfix([(OX.CONST, 0, 1.0), (OX.CONST, 0, nan), (OX.MAX, 0, 0), (OX.OUTPUT, 0, 0)], [], 1) == [1.0]
    # IEEE division by zero and the transcendental identities
    assert OX.eval_postfix([(OX.CONST, 0, -1.0), (OX.CONST, 0, 0.0), (OX.DIV, 0, 0), (OX.OUTPUT, 0, 0)], [], 1) == [-math.inf]
    v = OX.eval_postfix([(OX.INPUT, 0, 0), (OX.SIN, 0, 0), (OX.OUTPUT, 0, 0), (OX.INPUT, 0, 0), (OX.COS, 0, 0),
                         (OX.OUTPUT, 1, 0)], [0.7], 2)
    assert abs(v[0] ** 2 + v[1] ** 2 - 1.0) < 1e-15
    assert OX.eval_postfix([(OX.CONST, 0, 2.0), (OX.LOG, 0, 0), (OX.EXP, 0, 0), (OX.OUTPUT, 0, 0)], [], 1)[0] == \
        pytest.approx(2.0, rel=1e-15)
    with pytest.raises(ValueError):
        OX.eval_postfix([(OX.INPUT, 0, 0), (OX.INPUT, 0, 0), (OX.OUTPUT, 0, 0)], [1.0], 1)


@pytest.fixture(scope="module")
def apcg():
    import paper_2306_17801_amd as m

    m.load()
    return m


def test_compile_shares_common_subexpressions(apcg):
    from paper_2306_17801_amd.expr import Eval, Sym, sqrt

    x, y = Sym.inputs(2)
    s = x + y
    e = Eval([s * s, sqrt(s * s) + s], ninputs=2)
    st = e.stats()
    # x, y, x+y, (x+y)^2, sqrt, + : 6 instructions; x+y written 5 times (4
    # shared), s*s twice (1 shared)
    assert st["instructions"] == 6 and st["shared"] == 5 and st["folded"] == 0
    e.close()


def test_compile_folds_constants_and_exact_identities(apcg):
    from paper_2306_17801_amd.expr import Eval, Sym, const, sin, sqrt

    (x,) = Sym.inputs(1)
    # (2 + 3) * x: one folded constant, 3 instructions (const, x, mul)
    e = Eval([(const(2.0) + 3.0) * x], 1)
    assert e.stats() == {"instructions": 3, "folded": 1, "shared": 0}
    e.close()
    # x * 1, x / 1, x - 0, x + (-0), -(-x): all x itself
    e = Eval([x * 1.0, x / 1.0, x - 0.0, x + (-0.0), -(-x), 1.0 * x], 1)
    assert e.stats()["instructions"] == 1
    e.close()
    # x + 0 is not x for x = -0, so it stays; sin of a constant is not folded
    e = Eval([x + 0.0, sin(const(1.0))], 1)
    assert e.stats()["instructions"] == 5
    e.close()
    # sqrt(2) * sqrt(2) folds to the correctly rounded product, one constant
    e = Eval([sqrt(const(2.0)) * sqrt(const(2.0))], 0)
    assert e.stats()["instructions"] == 1
    e.close()


@pytest.mark.parametrize("tokens,nin,nout", [
    ([(20, 0, 0.0), (30, 0, 0.0)], 1, 1),                        # binary op on an empty stack
    ([(1, 0, 0.0), (1, 0, 0.0), (30, 0, 0.0)], 1, 1),             # a value left over
    ([(1, 3, 0.0), (30, 0, 0.0)], 2, 1),                          # input index out of range
    ([(2, 0, 1.0), (30, 0, 0.0), (2, 0, 2.0), (30, 0, 0.0)], 0, 1),  # output written twice
    ([(2, 0, 1.0), (30, 0, 0.0)], 0, 2),                          # output 1 never written
    ([(2, 0, 1.0), (99, 0, 0.0), (30, 0, 0.0)], 0, 1),            # unknown op
    ([(2, 0, 1.0), (30, 0, 0.0)], 0, 17),                         # too many outputs
])
def test_compile_rejects_malformed_programs(apcg, tokens, nin, nout):
    with pytest.raises(apcg.ApcgError) as e:
        apcg.apcg_expr_compile(tokens, nin, nout)
    assert e.value.code == apcg.APCG_ERR_INVALID_ARG


def test_compile_limits(apcg):
    # 129 distinct instructions exceed the register program's size
    toks = [(1, 0, 0.0)]
    for k in range(128):
        toks += [(2, 0, float(k + 1)), (20, 0, 0.0)]
    toks += [(30, 0, 0.0)]
    with pytest.raises(apcg.ApcgError):
        apcg.apcg_expr_compile(toks, 1, 1)
