"""MI355X-native fused coupled lattice Boltzmann sweep (flow, convection-
diffusion, vector magnetic) with the pair-wise moment, flux-increment and
moving-wall boundary schemes, behind the C ABI in include/lbm.h."""
from . import _lib  # noqa: F401
from .lbm import Lattice, build_links, lattice_table, params_from_scene  # noqa: F401

__all__ = ["Lattice", "build_links", "lattice_table", "params_from_scene"]
