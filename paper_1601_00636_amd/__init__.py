"""MI355X-native modulo-primes sieve for perfect cuboids (second cuboid
conjecture), after Gallyamov et al., arXiv:1601.00636.

The compute path lives in the HIP/C library `libcuboid.so` (sources in
`csrc/`, C interface in `include/cuboid.h`); `binding` is a thin ctypes layer
over it with the same function names.  `workloads` draws seeded inputs.
"""
__all__ = ["binding", "workloads"]


def __getattr__(name):
    if name == "binding":
        from . import binding
        return binding
    if name == "workloads":
        from . import workloads
        return workloads
    raise AttributeError(name)
