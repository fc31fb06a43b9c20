"""MI355X-native D2Q37 thermal lattice Boltzmann step (propagate, bc, collide).

The compute path is the gfx950 library built from csrc/ (C ABI in include/lb.h);
``lb.LB`` is its Python binding.  ``workload`` builds the seeded synthetic
Rayleigh-Taylor initial conditions.
"""

from . import workload  # noqa: F401

__all__ = ["workload", "lb"]


def __getattr__(name):
    if name == "lb":
        import importlib
        return importlib.import_module(".lb", __name__)
    raise AttributeError(name)
