"""Seeded synthetic input generators shared by the oracle and the HIP path."""
from .graphs import (Graph, rmat_graph, uniform_out_graph, sources_uniform,
                     sources_by_degree, random_walk_plan, workload)

__all__ = ["Graph", "rmat_graph", "uniform_out_graph", "sources_uniform",
           "sources_by_degree", "random_walk_plan", "workload"]
