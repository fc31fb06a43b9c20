"""MI355X-native D2Q37 thermal lattice Boltzmann step (propagate, bc, collide).

The compute path is the gfx950 library built from csrc/ (C ABI in include/lb.h);
``lb.LB`` is its Python binding and ``adjoint.kinetic_energy`` the
differentiable run behind torch.autograd.  ``workload`` builds the seeded
synthetic Rayleigh-Taylor initial conditions.  ``lb`` and ``adjoint`` load on
first use (they need torch and the built library).
"""

from . import workload  # noqa: F401

__all__ = ["workload", "lb", "adjoint"]


def __getattr__(name):
    if name in ("lb", "adjoint"):
        import importlib
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
