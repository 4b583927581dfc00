"""Seeded synthetic inputs for the ANI-style potential: parameter tables,
random MLP weights, molecular geometries, water boxes and serving requests.

This package is shared by the FP64 oracle and by the HIP path's tests and
benchmark.  It holds only input *data* (shapes, constants, random draws);
none of the potential's arithmetic (cutoffs, symmetry functions, the MLP,
forces or integration) lives here.
"""
from .params import (AEVTable, MLPTable, aev_table, mlp_table, SPECIES7, SPECIES4,
                     MASS_AMU, feature_count)
from .geometry import (random_molecule, single_molecule, conformer_batch, water_box, System,
                       triclinic_system,
                       pack_molecules,
                       config_system, CONFIGS)
from .requests import poisson_requests, maxwell_boltzmann, Request

__all__ = [
    "AEVTable", "MLPTable", "aev_table", "mlp_table", "SPECIES7", "SPECIES4",
    "MASS_AMU", "feature_count", "random_molecule", "single_molecule", "pack_molecules", "conformer_batch", "water_box",
    "System", "triclinic_system", "config_system", "CONFIGS", "poisson_requests", "maxwell_boltzmann",
    "Request",
]
