"""MI355X-native commutator-free exponential time-propagators (CFETs).

The propagation path lives in the HIP/C++ shared library ``libcfet.so``
(sources in ``csrc/``, C-ABI in ``include/cfet.h``); ``binding`` marshals
arguments to it with ctypes and uses PyTorch only for device memory and
streams.  ``inputs`` builds seeded synthetic Hamiltonians and states.

Importing this package does not load the library; ``binding.load()`` (called
on first use) does, and raises if it is missing -- there is no CPU fallback.
"""
__all__ = ["binding", "inputs"]
