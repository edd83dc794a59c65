"""MARS (Mean-field Annealing from a Random State) on MI355X.

The solver lives in a HIP/C++ shared library with a C ABI (``include/mars.h``);
``paper_1907_05124_amd.mars`` is its thin Python binding and
``paper_1907_05124_amd.inputs`` makes seeded synthetic instances.
"""
