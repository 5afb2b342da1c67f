"""MI355X-native (gfx950) BigGraphVis hot path: streaming community detection,
count-min-sketch supergraph and ForceAtlas2 layout, as hand-written HIP kernels
behind a C ABI (include/bgv.h).  Importing the package loads libbgv.so; it raises if
the library has not been built."""
from ._lib import BgvError  # noqa: F401
from .api import (FA2Energy, batched, batched_workspace, bh_tree, community, community_passes,  # noqa: F401
                  community_resume,
                  draw_supernodes, fa2_energy, fa2_grad, fa2_layout, fa2_params, pack_graphs, pipeline,
                  supergraph, validate_edges)

__all__ = ["BgvError", "FA2Energy", "community", "community_passes", "community_resume", "supergraph", "fa2_layout", "fa2_energy",
           "fa2_grad", "fa2_params", "pipeline", "validate_edges", "batched", "batched_workspace", "pack_graphs",
           "draw_supernodes", "bh_tree"]
