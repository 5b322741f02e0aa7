"""MI355X (gfx950) FP64 evaluation of the power-flow mismatch equations and
their Jacobian for Newton power flow (Cui, Li & Fang, Section II), behind
the C ABI of libpf (include/pf.h).

Submodules load lazily so that the input generators (``synth``) can be used
without the compiled library.
"""

__all__ = ["Plan", "PFError", "PFResidual", "build"]


def __getattr__(name):
    if name == "Plan":
        from .api import Plan
        return Plan
    if name == "PFError":
        from .capi import PFError
        return PFError
    if name == "PFResidual":
        from .autograd import PFResidual
        return PFResidual
    if name == "build":
        from .build import build
        return build
    raise AttributeError(name)
