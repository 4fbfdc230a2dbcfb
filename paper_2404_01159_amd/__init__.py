"""MI355X-native TensorRVEA generation: HIP kernels behind a C ABI
(include/rvea.h, librvea.so) and a thin ctypes binding."""
from .rvea import (Run, Batch, batch_footprint, Params, default_params, footprint, lattice_divisions, RveaError,
                   LINEAR_MULTIMODAL, SPHERE_UNIMODAL, SPHERE_MULTIMODAL, POLICY_LQ, POLICY_D, POLICY_E,
                   OP_GA, OP_DE, OP_PSO, OP_CSO, OP_RAND, OPERATORS, RVEA_EUNSUPPORTED,
                   EXPORTS, LIB_PATH, indicator_footprint, hypervolume, expected_utility)

__all__ = ["Run", "Batch", "batch_footprint", "Params", "default_params", "footprint", "lattice_divisions", "RveaError",
           "LINEAR_MULTIMODAL", "SPHERE_UNIMODAL", "SPHERE_MULTIMODAL", "POLICY_LQ", "POLICY_D", "POLICY_E",
           "OP_GA", "OP_DE", "OP_PSO", "OP_CSO", "OP_RAND", "OPERATORS", "RVEA_EUNSUPPORTED",
           "EXPORTS", "LIB_PATH", "indicator_footprint", "hypervolume", "expected_utility"]
