"""Exact sparse KNN join (BF / IIB / IIIB) on AMD MI355X: HIP kernels behind a C ABI.

    from paper_1011_2807_amd import DeviceCSR, build_index, knn_join, knn_join_bf
"""
from .knnj import (DeviceCSR, HostCSR, Index, KnnjError, Mlp, build_index, knn_join, knn_join_blocked,  # noqa: F401
                   knn_join_bf, load_library, STAT_CANDIDATES, STAT_COMPLETION, STAT_FALLBACKS, STAT_POSTINGS,
                   STAT_COUNT)
