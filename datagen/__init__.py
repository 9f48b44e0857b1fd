"""Seeded synthetic inputs for the penalized-quantile-regression solver.

This package is shared by the FP64 oracle and by the GPU path as *data only*:
it draws random numbers and lays them out, and contains none of the solver's
arithmetic.  Every draw comes from the Philox4x32-10 counter-based generator
(Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11), addressed by (row, column, stream, config) so that any entry of any
matrix can be regenerated independently on the host or on the device.
"""
from .philox import philox4x32, uniform01, KAT
from .configs import (make_gaussian, make_genotype, genotype_columns,
                      genotype_maf_thresholds, GenotypeSpec, GaussianSpec,
                      SPECS)

__all__ = ["philox4x32", "uniform01", "KAT", "make_gaussian", "make_genotype",
           "genotype_columns", "genotype_maf_thresholds", "GenotypeSpec",
           "GaussianSpec", "SPECS"]
