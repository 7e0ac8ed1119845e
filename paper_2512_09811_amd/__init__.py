"""ppwin: MI355X-native frequency-window solver for the particle-hole polarization propagator.

The compute path is the HIP library libppwin.so (sources in csrc/, C ABI in
include/ppwin.h); this package only builds and binds it.
"""
from .binding import (Handle, Server, PPError, spectrum, response, inject_hip_error, default_options, lib, LIB_PATH, PP_OK, PP_EINVAL, PP_ENOMEM, PP_ENOTCONV,
                      PP_EUNSTABLE, PP_EDEVICE, PP_ENOTSUP, PP_EPENDING, PP_FP64, PP_FP32,
                      PP_FOLDED, PP_RIESZ, PP_ASYNC, PP_SPLIT_BF16, PP_REDUCED, PP_DEVICE_PTRS)

__all__ = ["Handle", "Server", "PPError", "spectrum", "response", "inject_hip_error", "default_options", "lib", "LIB_PATH", "PP_OK", "PP_EINVAL", "PP_ENOMEM",
           "PP_ENOTCONV", "PP_EUNSTABLE", "PP_EDEVICE", "PP_ENOTSUP", "PP_EPENDING", "PP_FP64", "PP_FP32",
           "PP_FOLDED", "PP_RIESZ", "PP_ASYNC", "PP_SPLIT_BF16", "PP_REDUCED", "PP_DEVICE_PTRS"]
