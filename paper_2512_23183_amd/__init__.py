"""MI355X (gfx950) state-vector simulator: the gate / expectation /
parameter-shift hot path of LogosQ (arxiv 2512.23183) as hand-written HIP
behind a C ABI (``libsv.so``).

Submodules:
  inputs  -- seeded synthetic workloads (gate lists, Pauli sums, states)
  sv      -- ctypes binding of the C ABI (loads the built library)

The binding is imported lazily so that importing ``inputs`` never needs the
GPU library.
"""

__all__ = ["inputs", "sv"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
