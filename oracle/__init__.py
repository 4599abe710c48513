"""CPU oracle for the CRISP query engine -- TEST INFRASTRUCTURE ONLY.

A plain, slow, deliberately obvious float64/integer implementation of what the
CRISP index build and query engine compute (Dimitropoulos et al., "CRISP:
Correlation-Resilient Indexing via Subspace Partitioning", Sections 3-5 and
Algorithm 1).  It is the reference the GPU engine is checked against.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it.  The GPU engine never imports, links or calls anything here, and
this package imports nothing from the engine: the two share only the seeded
input generators in ``synth``.

Modules
-------
build   -- correlation check, rotation, subspace k-means, CSR, sign codes
query   -- both query modes step by step (Algorithm 1) + patience + learned prefix
brute   -- exact k-nearest-neighbour ground truth
theory  -- the Guaranteed-Mode recall lower bound (Theorem 1)
mlp     -- reference forward/backward/Adam for the learned candidate budget
"""
from . import build, query, brute, theory, mlp  # noqa: F401
