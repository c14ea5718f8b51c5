"""Seeded synthetic workload generators (inputs only; no max-flow arithmetic)."""
from .graphs import (Graph, SEED_BASE, CONFIGS, from_pairs, from_arcs, grid2d4, grid2d8_seg,
                     grid3d6, layered, rmat, random_graph, make_config, stream_instance,
                     stream_arrivals, seg_lut)
