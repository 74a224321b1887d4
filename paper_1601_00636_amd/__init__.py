"""MI355X-native modulo-primes sieve for perfect cuboids (second cuboid
conjecture), after Gallyamov et al., arXiv:1601.00636.

The compute path lives in the HIP/C library `libcuboid.so` (sources in
`csrc/`, C interface in `include/cuboid.h`); `binding` is a thin ctypes layer
over it with the same function names.  `workloads` draws seeded inputs.
Import the submodules directly: `from paper_1601_00636_amd import binding`.
"""
