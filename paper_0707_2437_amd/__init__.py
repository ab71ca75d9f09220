"""MI355X (gfx950) lattice Boltzmann library for the variable-speed-of-sound
D2Q9 model of Buick & Cosgrove (Sec. 3, Eq. 5): Python binding of liblbm.so.

Importing the package does not load the library; the first Lattice does,
and raises LibraryNotBuilt if it is missing (there is no CPU fallback).
"""
from ._lib import LibraryNotBuilt, lib
from .pool import GRAPH, GROUPED, PERSISTENT, Pool
from .lattice import (DTYPE_NAMES, DTYPES, EDEVICE, EINVAL, ENOMEM, ENONFINITE, ESTATE, F16S, F32, F32S, F64,
                      MODEL_EQUILIBRIUM, MODEL_FORCING, OK, XBC_INLET_OUTLET, XBC_PERIODIC, Lattice, LBMError,
                      footprint_bytes)

__all__ = ["Lattice", "Pool", "GROUPED", "GRAPH", "PERSISTENT", "LBMError", "LibraryNotBuilt", "lib", "footprint_bytes", "DTYPES", "DTYPE_NAMES",
           "F64", "F32", "F32S", "F16S", "OK", "EINVAL", "ENOMEM", "EDEVICE", "ESTATE", "ENONFINITE",
           "MODEL_FORCING", "MODEL_EQUILIBRIUM", "XBC_PERIODIC", "XBC_INLET_OUTLET"]
