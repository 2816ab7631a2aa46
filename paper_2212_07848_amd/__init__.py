"""MI355X-native fluctuating Shan-Chen lattice Boltzmann (arXiv:2212.07848).

The compute path is the HIP library ``libfsc.so`` (C ABI in include/fsc.h);
this package is its ctypes binding.  PyTorch is optional and only used for
device memory and streams (``Lattice(..., stream=torch_stream,
buffers=(tensor_a, tensor_b))``).
"""
from ._lib import (FSC_E4, FSC_E8, FSC_FP32_SHIFTED, FSC_FP64, FSC_SK_AXIS, FSC_SK_RADIAL,
                   EXPORTS, Ensemble, FscError, Lattice, Params, Surrogate, device_copy,
                   field_sk, lib, linear_corr, linear_sk, linear_sk_radial, make_params, mfma_probe,
                   normals, philox, stack_scales, tile_shapes)

__all__ = ["FSC_E4", "FSC_E8", "FSC_FP32_SHIFTED", "FSC_FP64", "FSC_SK_AXIS", "FSC_SK_RADIAL",
           "EXPORTS", "Ensemble", "FscError", "Lattice", "Params", "Surrogate", "device_copy",
           "field_sk", "lib", "linear_corr", "linear_sk", "linear_sk_radial", "make_params", "mfma_probe",
           "tile_shapes", "stack_scales",
           "normals", "philox"]
