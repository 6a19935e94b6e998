"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package holds input generators only: smooth Gaussian-blob ensembles shaped
like the paper's weather ensemble (Sec. 6.1: 1000 members on a 250x352x20 grid),
vertex-pair draws and initial network parameters.  None of the dependence
measures or the network arithmetic lives here.
"""
from .ensemble import (CONFIGS, EnsembleConfig, blob_geometry, amplitudes,
                       make_ensemble, vertex_index, vertex_coords,
                       population_cov, population_rho)
from .draws import random_pairs, random_vertices, random_positions, ray_positions
from .netparams import NetLayout, make_net_params

__all__ = ["CONFIGS", "EnsembleConfig", "blob_geometry", "amplitudes",
           "make_ensemble", "vertex_index", "vertex_coords", "population_cov",
           "population_rho", "random_pairs", "random_vertices", "random_positions",
           "ray_positions", "NetLayout",
           "make_net_params"]
