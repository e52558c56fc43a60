"""GDSW two-level overlapping Schwarz preconditioner for MI355X (gfx950).

The compute path lives in the HIP/C++ shared library ``libgdsw.so`` built from
``csrc/``; ``binding`` is a thin ctypes layer over its C ABI.  Importing this
package does not load the library; ``binding.lib()`` does, and fails loudly if
it has not been built.
"""
__all__ = ["problems", "binding"]
