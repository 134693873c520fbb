"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package draws random numbers and nothing else: pulse amplitudes, field
offsets, quasi-static noise, Haar-random target unitaries and finite-difference
coordinates. It holds none of the method's arithmetic (no operators, no
Liouvillian, no exponentials, no products, no fidelity); each side builds those
itself from the scalars returned here.
"""
from .configs import (A_MAX, B_RANGE, T1_US, T2_US, haar_unitary, config0, config1_batch,
                      config1, config2, config3_four, config3_six, config4_targets,
                      small_case, hubbard3)

__all__ = ["A_MAX", "B_RANGE", "T1_US", "T2_US", "haar_unitary", "config0", "config1_batch",
           "config1", "config2", "config3_four", "config3_six",
           "config4_targets", "small_case", "hubbard3"]
