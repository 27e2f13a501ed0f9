"""MI355X-native component-based normal integration (gfx950 HIP library + ctypes binding)."""
from .binding import (NI_E_ARG, NI_E_DEVICE, NI_E_MODEL, NI_E_NOMEM, NI_E_NONFINITE, NI_E_NOTCONV, NI_E_SHAPE,
                      NI_OK, NI_ORTHO, NI_PERSP, Context, NIError, lib, make_camera, ni_params_default)

__all__ = ["Context", "NIError", "lib", "make_camera", "ni_params_default", "NI_OK", "NI_E_ARG", "NI_E_SHAPE",
           "NI_E_NONFINITE", "NI_E_NOMEM", "NI_E_DEVICE", "NI_E_NOTCONV", "NI_E_MODEL", "NI_ORTHO", "NI_PERSP"]
