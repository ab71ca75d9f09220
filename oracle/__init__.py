"""FP64 CPU oracle for the variable-speed-of-sound D2Q9 lattice Boltzmann step.

TEST INFRASTRUCTURE. Only the tests, the smoke check and the benchmark's
CPU-baseline leg load this package. The product library never does, and the
two share no code.
"""
from .lbmref import (Oracle, lattice, alpha, equilibrium, equilibrium_c2, source, load, set_threads, get_threads,
                     MODEL_FORCING, MODEL_EQUILIBRIUM, XBC_PERIODIC, XBC_INLET_OUTLET)

__all__ = ["Oracle", "lattice", "alpha", "equilibrium", "equilibrium_c2", "source", "load", "set_threads", "get_threads",
           "MODEL_FORCING", "MODEL_EQUILIBRIUM", "XBC_PERIODIC", "XBC_INLET_OUTLET"]
