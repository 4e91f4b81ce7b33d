"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

Trajectories only (analytic undulator, arc, uniform and 3-D wiggle motions, and
a channeling generator with multiple scattering and radiative loss) plus the
workload presets.  This package holds none of the radiation-integral
arithmetic and imports neither the oracle nor the HIP binding.
"""
from . import analytic, channeling, presets  # noqa: F401
from .channeling import ChannelingConfig  # noqa: F401


def build(force: bool = True):
    """Compile the C generator."""
    return channeling.build(force=force)
