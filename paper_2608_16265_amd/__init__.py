"""MI355X-native derivative evaluator for structured NLPs (arXiv 2608.16265).

Import :class:`ExaModel` to compile a model description (see the
``exa_modeling`` package) into gfx950 kernels and evaluate its callbacks on
torch device tensors.  The package needs the native library libexa.so built
in place (``python -m paper_2608_16265_amd.build_lib``); it has no fallback:
touching any of the names below without the library raises ImportError.
"""
__all__ = ["ExaModel", "ExaError", "ExaBatch", "LagrangianGradient"]


def __getattr__(name):
    # Load the native library on first use, so that the build script in this
    # package can run before the library exists.
    if name in ("ExaModel",):
        from .model import ExaModel
        return ExaModel
    if name == "ExaError":
        from ._lib import ExaError
        return ExaError
    if name == "ExaBatch":
        from .batch import ExaBatch
        return ExaBatch
    if name == "LagrangianGradient":
        from .adjoint import LagrangianGradient
        return LagrangianGradient
    raise AttributeError(name)
