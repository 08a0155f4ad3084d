"""MI355X-native Volterra-integral TDSE marcher (HIP kernels behind a C ABI).

``paper_2001_06113_amd.tdse`` is the Python binding of ``libtdse.so`` (built
in-tree by ``paper_2001_06113_amd.build``).  Importing the package itself
loads nothing; the binding raises if the library has not been built.
"""
__all__ = ["tdse", "build"]
