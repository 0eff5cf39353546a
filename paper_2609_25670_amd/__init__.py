"""MI355X-native multirate MRT lattice-Boltzmann hot path for thermosolutal
dendritic solidification: a HIP library (csrc/, C ABI in include/lbm.h) and
its ctypes binding (lbm.py)."""

from .lbm import Simulation, simulation_for, load, LIB_PATH, EXPORTS  # noqa: F401
