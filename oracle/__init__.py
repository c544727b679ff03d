"""CPU oracle for supernodal selected inversion: TEST INFRASTRUCTURE ONLY.

A plain, slow, float64/complex128 numpy implementation of what the HIP path
computes, written from the paper (Jacquelin, Lin, Jia, Zhao, Yang, "A
Left-Looking Selected Inversion Algorithm and Task Parallelism on Shared
Memory Systems", arXiv:1604.02528).  Only the tests, the smoke entry point and
the benchmark's CPU-baseline leg may import it; the product library never
does, and this package imports nothing from the product.

Modules
  symbolic  elimination tree, column counts, supernode partition, row sets
            C(K), canonical ancestor index maps (Section 2.1, Eq. (newset)).
  factor    unpivoted supernodal LDL^T and the normalized factors
            Lhat = L_{C,K} L_{K,K}^{-1}, Dt^{-1} = (L_KK D_K L_KK^T)^{-1}
            (Alg. 1 steps 1-2; LDL^T specialization of Section 2.3).
  selinv    selected inversion: the dense definition, Alg. 1 (pull form) and
            Alg. 2 (left-looking push form with D, O, I and ID updates).
  adjoint   gradient of a loss on the selected entries with respect to the
            stored values of A (not in the paper; plain matrix calculus).

Parity pins live in tests/ (marked "not gpu").  Every function states the
passage it follows.
"""

from . import symbolic, factor, selinv, adjoint  # noqa: F401
