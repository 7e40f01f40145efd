"""MI355X-native free-space spectral Ewald evaluation of stokeslet, stresslet and
rotlet sums (af Klinteberg, Shamshirgar & Tornberg, arXiv:1607.04808).

The computation lives in the HIP library ``lib/libfse.so`` (C ABI in
``include/fse.h``); :mod:`.fse` is its Python binding.
"""
from .fse import (FseError, Geometry, Plan, Params, bounding_box, choose_params,  # noqa: F401
                  error_estimates, eval_noalloc, freespace_solve, fse_sum, geometry, lib, make_params,
                  precompute_cache_stats, rotlet, stokeslet,
                  stresslet)
