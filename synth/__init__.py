"""Seeded synthetic inputs shared by the tests, the oracle checks and the bench."""
from .graphs import (Graph, csr_from_edges, sbm, sbm_by_degree, disjoint_cliques, cycle,
                     complete_bipartite, random_weighted, gaussian_mixture, knn_graph,
                     knn_mixture, knn_mixture_device, sbm_device, batched_sbm_params, dcsbm_device, learned_params,
                     learned_graph, graph_agreement)
