"""Seeded synthetic input generators shared by the oracle and the HIP path."""
from .graphs import (Graph, hub_graph, rmat_graph, uniform_out_graph, sources_uniform,
                     sources_by_degree, random_walk_plan, poisson_requests, workload)

__all__ = ["Graph", "hub_graph", "rmat_graph", "uniform_out_graph", "sources_uniform",
           "sources_by_degree", "random_walk_plan", "poisson_requests", "workload"]
