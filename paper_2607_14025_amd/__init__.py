"""MI355X (gfx950) Sternheimer chi0 apply: HIP kernels behind a C ABI (libstern.so) and a ctypes binding."""
from .stern import (System, Model, SternError, apply_chi0_many, basis_info, lib, STERN_OK, STERN_WARN_NOT_CONVERGED,
                    STERN_FP64, STERN_MIXED, STERN_GUESS_ZERO, STERN_GUESS_LEARNED, STERN_GUESS_LEARNED_K,
                    STERN_GUESS_PREVIOUS,
                    STERN_INNER_PROJECTED, STERN_INNER_SHIFTED, EXPORTED)
