"""The oracle (test infrastructure only): plain CPU counting of embeddings.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP library.
"""
from .oracle import Prepared, count, count_per_root, list_embeddings, build, LIB_PATH

__all__ = ["Prepared", "count", "count_per_root", "list_embeddings", "build", "LIB_PATH"]
