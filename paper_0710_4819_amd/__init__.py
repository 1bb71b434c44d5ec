"""libacbm: adaptive cost block matching motion estimation on MI355X (gfx950).

The compute path is the HIP library ``libacbm.so`` built from ``csrc/``; the
Python side (``acbm``) only marshals arguments to its C ABI.  Importing this
package loads nothing; the first call through ``acbm`` loads the library and
raises if it has not been built.
"""
__all__ = ["acbm", "synth"]
__version__ = "0.1.0"
