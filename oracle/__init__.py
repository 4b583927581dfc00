"""FP64 CPU oracle for the ANI-style symmetry-function potential.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP library
(the only common module is ``workloads``, which holds input data and no
arithmetic of the method).

What it computes (the paper names the workload but prints no formula: the
ANI family's atom-centered symmetry functions, neighbor lists and per-element
networks, Methods "OpenMM-ML" and "Optimization Through NNPOps"; forces are
the negative energy gradient obtained by backpropagation, Methods "PyTorch
Model Support"):

* ``neighbors``  pair sets under the float32 distance predicate;
* ``aev``        radial and angular atomic environment vectors;
* ``mlp``        per-element networks with CELU, energies and their adjoint;
* ``potential``  energy per molecule, analytic forces, weight gradients,
                 the mean over an ensemble of networks, and a subset of a
                 larger system (mechanical embedding);
* ``integrator`` velocity-Verlet and LF-Middle Langevin MD in eV, A, amu, fs;
* ``rng``        the Philox4x32-10 counter-based generator and Box-Muller.

Every function is plain float64 NumPy with no blocking or fusion.
"""
from .neighbors import pair_list, pair_list_loops
from .aev import aev, aev_backward, pair_block_index, n_features
from .mlp import celu, celu_grad, mlp_forward, mlp_backward_input, mlp_weight_grads
from .potential import (energy_forces, energy, weight_gradients, EFResult,
                        ensemble_energy_forces, subset_energy_forces)
from .integrator import velocity_verlet, kinetic_energy, langevin_middle
from .rng import philox4x32_10, atom_normals

__all__ = [
    "pair_list", "pair_list_loops", "aev", "aev_backward", "pair_block_index",
    "n_features", "celu", "celu_grad", "mlp_forward", "mlp_backward_input",
    "mlp_weight_grads", "energy_forces", "energy", "weight_gradients", "EFResult",
    "ensemble_energy_forces", "subset_energy_forces",
    "velocity_verlet", "kinetic_energy", "langevin_middle", "philox4x32_10", "atom_normals",
]
