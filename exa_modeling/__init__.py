"""Model description and seeded synthetic workloads for structured NLPs.

This package is the *input* side of the project: it lets a modeler state an
NLP in the pattern-over-data form of the paper (Sec. 2.2, eq. simd) and it
draws the seeded synthetic instances used by the tests and the benchmark.

It performs none of the method's arithmetic: no evaluation, no
differentiation, no simplification and no sparsity analysis happen here.
Expressions are recorded exactly as written (``x**2`` stays a power node)
and handed over as a post-order node list plus data columns.  Both the
evaluator library and the CPU oracle consume that description, each with
its own implementation of everything downstream.
"""
from .ir import (Expr, Model, Pattern, VarBlock, ParBlock, DataSet, Node,
                 UNARY_OPS, BINARY_OPS, LEAF_OPS)
from . import ir as ops  # noqa: F401  (ops.exp, ops.sin, ...)
from .ir import (exp, log, sin, cos, tan, atan, sinh, cosh, tanh, sqrt, inv,
                 abs2, log1p, expm1)
from .twostage import TwoStageModel

__all__ = ["Expr", "Model", "Pattern", "VarBlock", "ParBlock", "DataSet",
           "Node", "UNARY_OPS", "BINARY_OPS", "LEAF_OPS", "exp", "log", "sin",
           "cos", "tan", "atan", "sinh", "cosh", "tanh", "sqrt", "inv", "abs2",
           "log1p", "expm1", "TwoStageModel"]
