"""MI355X-native many-body dispersion (MBD) energy and gradients.

Thin Python binding of ``libmbd_hip.so`` (C ABI in ``include/mbd.h``): the
functions below carry the C names and only marshal arguments (torch device
tensors -> device pointers, the current torch stream -> the HIP stream).  Every
step of the computation runs in the HIP kernels of the library; if the library
is missing, importing the binding functions raises.
"""
import ctypes
import os

from . import _abi
from ._abi import (MBD_OK, MBD_ERR_INVALID_ARGUMENT, MBD_ERR_NEGATIVE_EIGENVALUE,
                   MBD_ERR_NOT_CONVERGED, MBD_ERR_OUT_OF_MEMORY, MBD_ERR_DEVICE,
                   MBD_ERR_UNSUPPORTED, MBD_FP64, MBD_FP32_REFINED, MBD_PARAM_OMEGA,
                   MBD_PARAM_C6, MBD_WANT_ENERGY, MBD_WANT_GRAD_COORDS, MBD_WANT_GRAD_ALPHA0,
                   MBD_WANT_GRAD_OMEGA, MBD_WANT_GRAD_RVDW, MBD_WANT_GRAD_LATTICE,
                   MBD_WANT_EIGVALS, MBD_WANT_ERRORS, MbdSystem, MbdResult, lib, library_path)

__all__ = [n for n in dir(_abi) if n.startswith("MBD_")] + [
    "MbdSystem", "MbdResult", "lib", "library_path",
    "mbd_create", "mbd_destroy", "mbd_set_stream", "mbd_evaluate", "mbd_evaluate_batch",
    "mbd_eigh", "mbd_autotune", "mbd_load_tuning", "mbd_last_error", "mbd_set_profiling",
    "mbd_get_profile", "mbd_check_dc_buffers",
]

mbd_create = _abi.mbd_create
mbd_destroy = _abi.mbd_destroy
mbd_set_stream = _abi.mbd_set_stream
mbd_evaluate = _abi.mbd_evaluate
mbd_evaluate_batch = _abi.mbd_evaluate_batch
mbd_eigh = _abi.mbd_eigh
mbd_autotune = _abi.mbd_autotune
mbd_load_tuning = _abi.mbd_load_tuning
mbd_last_error = _abi.mbd_last_error
mbd_set_profiling = _abi.mbd_set_profiling
mbd_get_profile = _abi.mbd_get_profile
mbd_check_dc_buffers = _abi.mbd_check_dc_buffers
