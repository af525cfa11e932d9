"""MI355X-native MLCC3 triples hot path (right/left Jacobian transforms, ground-state
triples residual) behind the C-ABI library ``libmlcc3.so``.

Importing the package does not load the GPU library; ``paper_2202_08612_amd.mlcc3``
does, and raises if it has not been built.
"""
__all__ = ["inputs"]
