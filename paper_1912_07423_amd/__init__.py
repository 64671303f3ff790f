"""MI355X (gfx950) clock-driven spiking-network simulator built around work queues
(Bautembach et al., "Faster and Simpler SNN Simulation with Work Queues").

The simulation runs in hand-written HIP kernels behind the C ABI of include/snn.h
(libsnn.so); `Network` (one network) and `Batch` (many independent networks in one
persistent launch) are its Python binding.  `workloads` holds the synthetic network
descriptions.
"""
__all__ = ["Network", "Batch", "SnnError", "library_path", "memory_cache_stats", "memory_cache_release"]


def __getattr__(name):
    if name == "Network":
        from .network import Network
        return Network
    if name == "Batch":
        from .network import Batch
        return Batch
    if name in ("memory_cache_stats", "memory_cache_release"):
        from . import network
        return getattr(network, name)
    if name == "SnnError":
        from ._lib import SnnError
        return SnnError
    if name == "library_path":
        from ._lib import LIB_PATH
        return LIB_PATH
    raise AttributeError(name)
