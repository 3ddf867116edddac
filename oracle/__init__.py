"""CPU oracle for the space-switching BGV hot path.

TEST INFRASTRUCTURE ONLY: this package exists to check the GPU library.  Only the
test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import it; the product path never does.  It shares no code with the GPU
library: it derives its own primes, roots, slot structure and polynomial tables,
and computes every ring product with the schoolbook definition in exact integer
arithmetic (``ring.c``).
"""
