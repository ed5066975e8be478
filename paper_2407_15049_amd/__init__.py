"""MI355X (gfx950) low-rank SDP hot path: C-ABI HIP library + ctypes binding.

The library ``_lib/liblrsdp.so`` is built by ``__graft_entry__.build()``; the
binding lives in ``paper_2407_15049_amd.lrsdp``.
"""

__all__ = ["lrsdp"]
