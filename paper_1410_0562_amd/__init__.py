"""set-bwte on MI355X: incremental BWT of a DNA string set, built per block on
the GPU (Pantaleoni, arXiv:1410.0562, Algorithm 1).

The GPU library is ``libbwtset.so`` (C ABI declared in ``include/bwtset.h``);
``paper_1410_0562_amd.bwtset`` is its Python binding.  Importing this package
loads nothing; the binding loads the library on first use and raises if it has
not been built.
"""

__all__ = ["bwtset", "synth"]
