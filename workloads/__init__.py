"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark. This package holds input recipes only (initial velocity fields,
rotor geometry and polar tables, turbine trees); it contains none of
the lattice-Boltzmann or actuator-line arithmetic."""
from .fields import tgv_field, shear_wave_field, random_phase_field, shell_spectrum
from .rotor import (make_rotor, synthetic_polars, single_turbine_rotor, turbine_row_rotors,
                    turbine_row_inflow)
from . import turbines

__all__ = ["tgv_field", "shear_wave_field", "random_phase_field", "shell_spectrum",
           "make_rotor", "synthetic_polars", "single_turbine_rotor",
           "turbine_row_rotors", "turbine_row_inflow", "turbines"]
