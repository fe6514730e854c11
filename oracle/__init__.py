"""CPU FP64 oracle of the linear bond-based peridynamic model (test infrastructure only).

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg import
this package.  The product library never does, and the two share no code.
"""
from .oracle import (Problem, adr, adr_density, adr_step, all_bonds, alpha_2d, alpha_3d, apply, assemble_dense, bond_stretch,  # noqa: F401
                     broken_csr, crack_update,
                     build_oracle, crack_to_bonds, energy, energy_parts, fft_apply, fft_setup, force, grad_cg, grad_dense, lifted_rhs,
                     generating_blocks, periodic_apply, precond_apply, precond_apply_periodic,
                     precond_symbol, solve_cg, solve_dense, surface_volume_factors, vv)
