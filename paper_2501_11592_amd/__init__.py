"""MI355X-native CLOMP hot path (arXiv 2501.11592): C-ABI library + thin binding.

Importing the package loads nothing native; the HIP library is opened on the
first call through `paper_2501_11592_amd.clomp` (and fails loudly if it has not
been built).
"""

__all__ = ["clomp", "workloads"]
