"""MI355X-native KMV wave propagation: forward, adjoint and gradient of the
time-domain FWI misfit with mass-lumped KMV finite elements (HIP for gfx950
behind a C ABI; this package is the Python binding).

    from paper_2108_10946_amd import Mesh, Problem
    mesh = Mesh(coords, cells, degree=4)
    prob = Problem(mesh, dt, n_steps, precision="fp32")
    prob.set_sources([[4.0, 0.01]], f0=5.0, t0=0.2)
    prob.set_receivers(receivers)
    traces = prob.forward(c)                       # c: float64 cuda tensor, DOF order
    J, grad, traces = prob.misfit_gradient(c, observed)
    result = invert(library_objective([prob], [observed]), c0, mesh.lumped_mass())  # Algorithm 1
"""
from .kmvwave import (KMVError, KMV_FP32, KMV_FP64, kmv_element_tables, lib)
from .api import Mesh, Problem, Server
from .autograd import FWIMisfit, fwi_misfit
from .fwi import InversionResult, invert, library_objective

__all__ = ["Mesh", "Problem", "Server", "FWIMisfit", "fwi_misfit", "invert", "library_objective",
           "InversionResult", "KMVError", "KMV_FP32", "KMV_FP64", "kmv_element_tables", "lib"]
