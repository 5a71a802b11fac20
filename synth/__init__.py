"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only builds *inputs*: simplicial meshes, P-wavespeed models, damping
profiles and acquisition layouts.  It holds none of the method's arithmetic (no
element tables, no operators, no time stepping, no wavelet), so the oracle and the
HIP path can both draw their inputs from it without sharing any computation.
"""
from .meshes import (structured_tri, nvb_graded_tri, jitter_vertices, kuhn_tet_box,
                     graded_tet_box, mesh_quality_tri)
from .models import (layered_anomaly_vp, homogeneous_vp, sponge_eta, surface_receivers,
                     surface_sources, grid_receivers_3d, layered_anomaly_vp_3d,
                     sponge_eta_3d)
from . import configs
