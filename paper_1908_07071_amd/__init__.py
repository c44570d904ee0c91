"""MI355X-native LOR-Schwarz preconditioned CG for high-order CG / IP / BR2-DG Poisson.

The solver lives in the HIP library ``liblor.so`` (C ABI: include/lor.h);
``paper_1908_07071_amd.lor`` is its ctypes binding and
``paper_1908_07071_amd.inputs`` generates seeded synthetic problem data.
Importing the package itself loads nothing.
"""
