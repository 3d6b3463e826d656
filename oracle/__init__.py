"""FP64 CPU oracle of the online tensor method (Huang, Niranjan, Hakeem,
Anandkumar, "Online Tensor Methods for Learning Latent Variable Models").

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package.  The product path (the HIP library
and its Python binding) never imports, links or calls it, and shares no code,
header, table or helper with it.  The only common dependency is the seeded
input generator module, which holds none of the method's arithmetic.

Everything here is plain numpy/scipy in float64, written from the paper's
equations in the paper's order, with library primitives (matmul, sparse
matmul, eigh, svd) as steps and no blocking, fusion or reordering.
"""
from .otm import *  # noqa: F401,F403

