"""MI355X-native patch-based quadtree AMR advance + ghost fill (arXiv:1703.03116).

The compute path is the HIP library libfcmi.so (C ABI in include/fc.h);
``binding`` marshals arguments to it with PyTorch device memory.
"""
from .metrics import cell_updates, cell_update_rate, stable_dt  # noqa: F401

__all__ = ["binding", "metrics"]
