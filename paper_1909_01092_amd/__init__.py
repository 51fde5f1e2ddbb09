"""MI355X-native fluctuating two-component D3Q19 lattice Boltzmann step with a
settling wettable sphere (Xue, Biferale, Sbragaglia, Toschi, "A lattice
Boltzmann study of particle settling in a fluctuating multicomponent fluid
under confinement").

The compute path is the HIP library liblbm.so (C ABI: include/lbm.h); this
package only marshals arguments to it.
"""
from . import workloads  # noqa: F401

__all__ = ["Simulation", "workloads", "workspace_bytes"]


def __getattr__(name):
    if name in ("Simulation", "workspace_bytes", "make_params"):
        from . import sim
        return getattr(sim, name)
    raise AttributeError(name)
