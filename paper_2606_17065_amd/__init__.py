"""MI355X (gfx950) mixture-of-experts layer: hand-written HIP kernels behind
a C ABI (include/moe.h), with a thin ctypes binding.

Submodules load lazily: ``synth`` (seeded inputs) imports nothing else;
``_lib`` loads libmoe.so on first use and raises if it is missing; ``layer``
wraps the ABI for torch device tensors.
"""
