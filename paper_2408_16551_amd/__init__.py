"""MI355X-native polyphase filter bank channelizer (HIP for gfx950).

The compute path lives in the C-ABI shared library ``libtina_pfb.so`` built
from ``csrc/``; ``pfb`` is a thin ctypes binding over it.  Importing this
package does not load the library: the binding loads it on first use and
raises if it is missing, so there is no CPU fallback.
"""
__all__ = ["pfb", "workloads"]
