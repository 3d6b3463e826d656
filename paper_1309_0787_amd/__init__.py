"""MI355X (gfx950) hot path of the online tensor method for latent variable
models: M2 operator, randomized whitener, whitening SpMM, STGD on the implicit
whitened third moment, and post-processing, behind the C ABI of libotm.so."""
from . import otm  # noqa: F401
