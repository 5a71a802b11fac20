"""Object wrappers over the same-name ctypes calls (marshalling only)."""
from __future__ import annotations

import numpy as np

from . import kmvwave as K


def _torch():
    import torch
    return torch


class Mesh:
    """A simplicial mesh discretised with KMV elements of one degree (host-side
    preprocessing: DOF numbering, patches, gather words, geometry, lumped mass)."""

    def __init__(self, coords, cells, degree, patch_cells=0):
        coords = np.asarray(coords, dtype=np.float64)
        self.dim = coords.shape[1]
        self.degree = degree
        self.handle = K.kmv_mesh_create(self.dim, degree, coords, cells, patch_cells)
        info = K.kmv_mesh_info(self.handle)
        self.n_dofs = info["n_dofs"]
        self.n_cells = info["n_cells"]
        self.n_nodes = info["n_nodes"]
        self.n_patches = info["n_patches"]
        self.n_shared_dofs = info["n_shared_dofs"]

    def dof_coords(self):
        return K.kmv_mesh_dof_coords(self.handle, self.dim)

    def lumped_mass(self):
        return K.kmv_mesh_lumped_mass(self.handle)

    def boundary_mass(self):
        """b_i = integral of phi_i over the mesh boundary (the absorbing term's weights)."""
        return K.kmv_mesh_boundary_mass(self.handle)

    def cell_dofs(self):
        return K.kmv_mesh_cell_dofs(self.handle)

    def cfl_dt(self, c):
        """Gershgorin step bound 2/sqrt(max_i sum_j |K_ij| / M_i) (host)."""
        return K.kmv_cfl_dt(self.handle, np.asarray(c, dtype=np.float64))

    def validate(self):
        K.kmv_mesh_validate(self.handle)

    def patch_stats(self, adjoint=False):
        """Most cells and shared refs in one patch, and the refs the step kernel
        finishes in its first batch (kmv_mesh_patch_stats)."""
        return K.kmv_mesh_patch_stats(self.handle, adjoint)

    def nodal_values(self, fn):
        x = self.dof_coords()
        return fn(*[x[:, r] for r in range(self.dim)])

    def close(self):
        if getattr(self, "handle", None):
            K.kmv_mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """Device state for n_shots shots on one mesh (see kmv_problem_create).

    With n_shots > 1 the shots share wave speed, damping, wavelet and receivers;
    sources are given shot-major, traces and observed data are
    [n_shots, n_steps, n_rec], and J and the gradient are sums over the shots.
    gradient_every = r > 1 subsamples the gradient pairing (and the stored
    forward states) every r steps, scaled by r."""

    def __init__(self, mesh: Mesh, dt, n_steps, precision="fp64", checkpoint_every=0, mem_budget=0,
                 n_shots=1, gradient_every=1):
        self.mesh = mesh
        self.dt = float(dt)
        self.n_steps = int(n_steps)
        self.n_shots = int(n_shots)
        self.precision = K.KMV_FP32 if precision in ("fp32", K.KMV_FP32) else K.KMV_FP64
        self.gradient_every = int(gradient_every)
        self.handle = K.kmv_problem_create(mesh.handle, self.precision, self.dt, self.n_steps,
                                           checkpoint_every, mem_budget, self.n_shots, self.gradient_every)
        self.n_rec = 0
        self.n_src = 0

    @property
    def dtype(self):
        torch = _torch()
        return torch.float32 if self.precision == K.KMV_FP32 else torch.float64

    def info(self):
        return K.kmv_problem_info(self.handle)

    def cfl_dt(self, c):
        return self.mesh.cfl_dt(c)

    def spectral_radius(self, c, iters=200, seed=0):
        return K.kmv_spectral_radius(self.handle, self._c(c), iters, seed)

    def set_damping(self, eta):
        K.kmv_set_damping(self.handle, eta)

    def set_pml(self, sigma):
        """Perfectly matched layer with damping functions sigma [n_dofs, dim] (DOF
        order; one column per axis), or None to turn it off (kmv_set_pml)."""
        if sigma is not None and len(sigma) != self.mesh.n_dofs:
            raise ValueError("sigma must hold the mesh's n_dofs rows")
        K.kmv_set_pml(self.handle, sigma, self.mesh.dim)

    def set_absorbing_boundary(self, enable=True):
        """First-order absorbing boundary on every boundary facet (du/dt + c du/dn = 0),
        with its term in the gradient; off by default (homogeneous Neumann)."""
        K.kmv_set_absorbing_boundary(self.handle, enable)

    def set_sources(self, xs, f0=5.0, t0=None, amp=1.0):
        xs = np.asarray(xs, dtype=np.float64)
        xs = xs.reshape(-1, xs.shape[-1]) if xs.ndim == 3 else np.atleast_2d(xs)  # [n_shots, n, dim] or flat
        K.kmv_set_sources(self.handle, xs, f0, 1.0 / f0 if t0 is None else t0, amp)
        self.n_src = len(xs)

    def set_source_wavelet(self, w):
        """w: [n_steps] for every shot, or [n_shots, n_steps], one wavelet per shot."""
        w = np.asarray(w, dtype=np.float64)
        if w.ndim not in (1, 2) or w.shape[-1] != self.n_steps:
            raise ValueError(f"wavelet must be [n_steps] or [n_shots, n_steps] with n_steps = {self.n_steps}")
        if w.ndim == 2:
            if w.shape[0] != self.n_shots:
                raise ValueError(f"per-shot wavelets need {self.n_shots} rows, got {w.shape[0]}")
            K.kmv_set_source_wavelets(self.handle, w)
        else:
            K.kmv_set_source_wavelet(self.handle, w)

    def set_receivers(self, xr):
        xr = np.atleast_2d(np.asarray(xr, dtype=np.float64))
        K.kmv_set_receivers(self.handle, xr)
        self.n_rec = len(xr)

    def _shape(self, *tail):
        """Shape of a per-shot array: [n_steps, ...] for one shot, else [n_shots, n_steps, ...]."""
        return (self.n_steps, *tail) if self.n_shots == 1 else (self.n_shots, self.n_steps, *tail)

    def _c(self, c):
        torch = _torch()
        if not (isinstance(c, torch.Tensor) and c.is_cuda and c.dtype == torch.float64):
            raise TypeError("c must be a float64 CUDA tensor in DOF order")
        if c.numel() != self.mesh.n_dofs:
            raise ValueError("c has the wrong length")
        return c.contiguous()

    def forward(self, c, out=None):
        torch = _torch()
        c = self._c(c)
        tr = out if out is not None else torch.empty(self._shape(self.n_rec), dtype=self.dtype,
                                                      device=c.device)
        if tr.numel() != self.n_shots * self.n_steps * self.n_rec or not tr.is_contiguous():
            raise ValueError("out must be a contiguous " + str(self._shape(self.n_rec)) + " tensor")
        K.kmv_forward(self.handle, c, tr)
        return tr

    def misfit_gradient(self, c, observed, keep_traces=False):
        torch = _torch()
        c = self._c(c)
        obs = observed.to(dtype=self.dtype).contiguous()
        if tuple(obs.shape) != self._shape(self.n_rec):
            raise ValueError("observed must be " + str(list(self._shape(self.n_rec))))
        g = torch.empty(self.mesh.n_dofs, dtype=torch.float64, device=c.device)
        tr = torch.empty_like(obs) if keep_traces else None
        J = K.kmv_misfit_gradient(self.handle, c, obs, g, tr)
        return J, g, tr

    def misfit(self, c, observed, keep_traces=False):
        """J only (forward solve + float64 misfit, no adjoint sweep)."""
        torch = _torch()
        c = self._c(c)
        obs = self._observed(observed)
        tr = torch.empty_like(obs) if keep_traces else None
        J = K.kmv_misfit(self.handle, c, obs, tr)
        return (J, tr) if keep_traces else J

    def misfit_gradient_accumulate(self, c, observed, J_acc, grad_acc):
        """J_acc + J, and grad_acc (float64 CUDA tensor) += dJ/dc in the library."""
        torch = _torch()
        c = self._c(c)
        obs = self._observed(observed)
        if not (isinstance(grad_acc, torch.Tensor) and grad_acc.is_cuda and grad_acc.dtype == torch.float64
                and grad_acc.numel() == self.mesh.n_dofs and grad_acc.is_contiguous()):
            raise TypeError("grad_acc must be a contiguous float64 CUDA tensor of n_dofs values")
        return K.kmv_misfit_gradient_accumulate(self.handle, c, obs, float(J_acc), grad_acc)

    def status(self):
        """Synchronise and raise KMVError (KMV_ECFL / KMV_ENUMERIC) if the most recent
        solve went non-finite (kmv_problem_status)."""
        K.kmv_problem_status(self.handle)

    def _observed(self, observed):
        obs = observed.to(dtype=self.dtype).contiguous()
        if tuple(obs.shape) != self._shape(self.n_rec):
            raise ValueError("observed must be " + str(list(self._shape(self.n_rec))))
        return obs

    def adjoint(self, c, adj, keep_lambda=False, src_trace=False):
        torch = _torch()
        c = self._c(c)
        adj = adj.to(dtype=self.dtype).contiguous()
        if tuple(adj.shape) != self._shape(self.n_rec):
            raise ValueError("adj must be " + str(list(self._shape(self.n_rec))))
        if keep_lambda and self.n_shots != 1:
            raise ValueError("keep_lambda needs a one-shot problem")
        lam = (torch.empty((self.n_steps + 1, self.mesh.n_dofs), dtype=self.dtype, device=c.device)
               if keep_lambda else None)
        st = (torch.empty(self._shape(self.n_src // self.n_shots), dtype=self.dtype, device=c.device)
              if src_trace else None)
        K.kmv_adjoint(self.handle, c, adj, lam, st)
        return lam, st

    def stiffness_apply(self, c, u):
        torch = _torch()
        c = self._c(c)
        u = u.to(dtype=self.dtype).contiguous()
        y = torch.empty_like(u)
        K.kmv_stiffness_apply(self.handle, c, u, y)
        return y

    def close(self):
        if getattr(self, "handle", None):
            K.kmv_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Shot server on the current device: requests are admitted in arrival order
    as slots and device memory free up, and run concurrently, each on its own
    stream (see kmv_server_create).  A request is one shot (xs [n_src, dim]) or
    several sharing the rest (xs [n_shots, n_src, dim], observed and traces
    [n_shots, n_steps, n_rec], J and grad summed over the shots), which run as one
    multi-shot problem.  Inputs are host arrays; the results come back as host
    arrays."""

    def __init__(self, mem_budget=0, max_slots=4):
        self.handle = K.kmv_server_create(mem_budget, max_slots)
        self._prec = {}
        self._keep = {}  # meshes of pending requests stay alive

    def submit(self, mesh: Mesh, c, xs, xr, dt, n_steps, precision="fp32", eta=None, observed=None,
               forward_only=False, f0=5.0, t0=None, amp=1.0, absorbing=False, wavelets=None):
        """wavelets: None (Ricker of f0, t0, amp) or [n_shots, n_steps], one per shot."""
        prec = K.KMV_FP64 if precision == "fp64" else K.KMV_FP32
        t = K.kmv_server_submit(self.handle, mesh.handle, prec, dt, n_steps, c, xs, xr, f0,
                                1.0 / f0 if t0 is None else t0, amp, eta=eta, observed=observed,
                                forward_only=forward_only, absorbing=absorbing, wavelets=wavelets)
        self._prec[t] = prec
        self._keep[t] = mesh
        return t

    def poll(self, ticket):
        """None while pending, else a dict (status, J, traces, grad, timestamps)."""
        return K.kmv_server_poll(self.handle, ticket, self._prec[ticket])

    def wait(self, ticket, timeout=-1.0):
        return K.kmv_server_wait(self.handle, ticket, self._prec[ticket], timeout)

    def release(self, ticket):
        K.kmv_server_release(self.handle, ticket)
        self._prec.pop(ticket, None)
        self._keep.pop(ticket, None)

    def result(self, ticket):
        """Wait for a request, return its results and free them in the library."""
        r = self.wait(ticket)
        self.release(ticket)
        return r

    def stats(self):
        return K.kmv_server_stats(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            K.kmv_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
