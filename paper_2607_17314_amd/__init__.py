"""ISDF-xTC hot path on MI355X: Python binding of libisdfxtc (include/isdf_xtc.h).

The package holds the HIP sources (csrc/), their build (build.py) and the
binding (api.py). Loading the binding does not touch the GPU; calls need the
built library and a visible GPU, and raise if either is missing.
"""
from ._lib import (XTC_D1, XTC_D4, XTC_ESCALE, XTC_FIELD, XTC_FIT_XI, XTC_FIT_XIGRAD, XTC_FP64,
                   XTC_SELECT_LEARNED, XTC_SELECT_LEARNED_JUDGED, XTC_SELECT_QR, XTC_SPLIT_F16,
                   XTC_U1, XTC_U3, XTC_ULAP, XTC_U_BH, XTC_U_EE, lib)

__all__ = ["lib", "XTC_U1", "XTC_U3", "XTC_ULAP", "XTC_D1", "XTC_D4", "XTC_FIELD", "XTC_ESCALE",
           "XTC_FP64", "XTC_SPLIT_F16", "XTC_U_EE", "XTC_U_BH", "XTC_SELECT_QR",
           "XTC_SELECT_LEARNED", "XTC_SELECT_LEARNED_JUDGED", "XTC_FIT_XI", "XTC_FIT_XIGRAD"]
