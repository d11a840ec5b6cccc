"""lbgrid: MI355X-native over-decomposed grid update with per-chunk load
measurement and chunk-to-slot rebalancing (after arXiv 1310.4218).

Importing the package loads nothing; the HIP library is opened on first use by
``paper_1310_4218_amd.grid`` and the call fails loudly if it is missing.
"""
__all__ = ["workloads"]
