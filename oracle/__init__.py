"""FP64 CPU oracle for the consistent neural message-passing layer.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call
or execute anything here; only the tests, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the GPU path: it builds its own
graphs from the mesh (Sec. II-A) and evaluates the paper's equations in plain
NumPy float64, literally and without blocking, fusion or reordering.

Modules
-------
graph  distributed graph generation from a spectral-element mesh (Sec. II-A,
       Figs. 2-4): reduced sub-graphs, edge and node degrees, halo lists.
nmp    the consistent NMP layer (Eq. 4a-e), the encode-process-decode model
       (Sec. III), the losses (Eq. 5, Eq. 6a-c) and a hand-written reverse
       mode for all of them.
ball   exact evaluation of single output nodes on their receptive fields,
       for parity checks at sizes where a whole-graph evaluation is too slow.

Pinned by tests/test_oracle_*.py against GLL closed forms, exact integer
sums, brute-force loops, the paper's Table I/II numbers, R-consistency
(Eq. 2, 3), adjoint dot-product identities and central finite differences.
"""
