"""ORACLE -- test infrastructure only.

Plain FP64 CPU implementation of one step of appearance-driven simplification
(Hasselgren et al.), used to check the GPU path.  Only tests, the smoke check
and the benchmark's CPU-baseline leg may import it; the product path never
does, and the two share no code.
"""
