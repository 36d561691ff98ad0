"""TENO-D gas-kinetic scheme (arXiv:2309.10534) on MI355X.

The compute path lives in the HIP library ``libtgks.so`` behind the C ABI of
``include/tgks.h``; ``paper_2309_10534_amd.tgks`` binds it.  Importing this
package loads nothing: the library is opened on first use and a missing
library is an error, never a fallback.
"""
__all__ = ["inputs"]
