"""CPU oracle of the Wilson hopping operator -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 implementations used to check the HIP path.  Only the tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
anything from this package; the product path never does.
"""
