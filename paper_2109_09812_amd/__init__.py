"""meshrx: GPU re-indexing of indexed meshes (duplicate- and unused-vertex
removal) for AMD MI355X, after Wald's parallel re-indexing method (sort,
run-head flags, prefix sums, scatters, index remap).

The compute lives in libmeshrx.so (hand-written HIP for gfx950, C ABI in
include/meshrx.h); this package only marshals arguments.
"""
from ._lib import (MRX_TUNING_BANDS, MRX_TUNING_CLAIMED_TILES, MRX_TUNING_HASH_GROUPS, MRX_TUNING_SORT_ALL,  # noqa: F401
                   MRX_TUNING_WIDE_LOOKBACK, MeshrxError, load, tunings)

__all__ = ["MRX_TUNING_CLAIMED_TILES", "MRX_TUNING_WIDE_LOOKBACK", "MRX_TUNING_SORT_ALL", "MRX_TUNING_HASH_GROUPS",
           "MRX_TUNING_BANDS",
           "MeshrxError", "load", "tunings",
           "reindex_mesh", "reindex_mesh_noalloc", "reindex_mesh_batched", "merge_meshes", "extract_submesh",
           "gather_attrs", "GatherAttrs", "BatchedReindexer", "GraphedBatchedReindexer",
           "Reindexer", "MeshMerger", "SubmeshExtractor", "workspace_size"]


def __getattr__(name):
    # torch-dependent API is imported on first use
    if name in ("reindex_mesh", "reindex_mesh_noalloc", "reindex_mesh_batched", "merge_meshes", "extract_submesh", "Extracted",
                "MeshMerger", "SubmeshExtractor",
                "gather_attrs", "GatherAttrs",
                "BatchedReindexer", "GraphedBatchedReindexer", "workspace_size", "Reindexed", "Reindexer",
                "BatchReindexed"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
