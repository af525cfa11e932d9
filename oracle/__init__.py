"""CPU oracle for the MLCC3 triples hot path (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path.
Functions without an independent pin are marked "parity unpinned" in their
docstrings.
"""
