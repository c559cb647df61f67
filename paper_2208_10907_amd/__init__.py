"""MI355X-native H^2-ULV dense direct solver (arXiv 2208.10907).

The factorization and solve run in the HIP library built from ``csrc/``; this
package holds only its Python binding (``h2ulv``) and the build script.
"""
from . import h2ulv  # noqa: F401
from .h2ulv import (H2ULVError, Factor, Structure, factorize, factorize_batch,  # noqa: F401
                    make_params, params_from_problem)
