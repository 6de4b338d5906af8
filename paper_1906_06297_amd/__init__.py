"""MI355X (gfx950) checkerboard Metropolis simulation of the 2D Ising model.

The hot path lives in hand-written HIP kernels behind the C ABI of
``libising.so`` (include/ising.h); this package is the thin Python binding.
"""
from ._lib import IsingError, load  # noqa: F401
from .lattice import (ARNet, Batch, GlassBonds, Lattice, MatmulLattice, batch_sweep_noalloc,  # noqa: F401
                      arnet_num_params, batch_words, mh_independence, set_sweep_kernel,
                      spins_minibatch,
                      spins_observables, thresholds, words_per_colour)
