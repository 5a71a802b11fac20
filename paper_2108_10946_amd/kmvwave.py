"""ctypes binding of the kmvwave C ABI (include/kmvwave.h), same names.

Argument marshalling only: every numerical step runs in the HIP library
``libkmvwave.so`` next to this file.  If the library is missing, importing the
binding works but the first call raises ``RuntimeError`` (there is no fallback).

Device buffers are torch tensors on the current HIP device (torch is used for
device memory and streams only); the stream is torch's current stream unless one
is passed.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkmvwave.so")

KMV_OK, KMV_EINVAL, KMV_ENOMEM, KMV_EDEGREE, KMV_EMESH = 0, -1, -2, -3, -4
KMV_EOUTSIDE, KMV_ECFL, KMV_ENUMERIC, KMV_EDEVICE, KMV_EBUSY, KMV_ESTATE = -5, -6, -7, -8, -9, -10
KMV_FP64, KMV_FP32 = 0, 1

ERROR_NAMES = {0: "KMV_OK", -1: "KMV_EINVAL", -2: "KMV_ENOMEM", -3: "KMV_EDEGREE", -4: "KMV_EMESH",
               -5: "KMV_EOUTSIDE", -6: "KMV_ECFL", -7: "KMV_ENUMERIC", -8: "KMV_EDEVICE",
               -9: "KMV_EBUSY", -10: "KMV_ESTATE"}

# every symbol include/kmvwave.h declares
DECLARED = [
    "kmv_last_error", "kmv_element_tables", "kmv_mesh_create", "kmv_mesh_info",
    "kmv_mesh_dof_coords", "kmv_mesh_lumped_mass", "kmv_mesh_boundary_mass", "kmv_mesh_cell_dofs", "kmv_mesh_validate",
    "kmv_mesh_patch_stats",
    "kmv_mesh_destroy",
    "kmv_problem_create", "kmv_cfl_dt", "kmv_spectral_radius", "kmv_set_damping", "kmv_set_pml", "kmv_set_absorbing_boundary",
    "kmv_set_sources", "kmv_set_source_wavelet", "kmv_set_source_wavelets", "kmv_set_receivers", "kmv_forward",
    "kmv_forward_noalloc", "kmv_misfit_gradient", "kmv_misfit_gradient_accumulate", "kmv_misfit", "kmv_problem_status", "kmv_adjoint", "kmv_stiffness_apply", "kmv_problem_info", "kmv_problem_num_shots",
    "kmv_profile_enable", "kmv_profile_read", "kmv_problem_destroy",
    "kmv_server_create", "kmv_server_submit", "kmv_server_poll", "kmv_server_wait",
    "kmv_server_release", "kmv_server_stats", "kmv_server_destroy",
]


class KMVError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class kmv_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("dt", C.c_double), ("n_steps", C.c_int64),
                ("checkpoint_every", C.c_int64), ("mem_budget", C.c_size_t), ("n_shots", C.c_int),
                ("gradient_every", C.c_int64)]


class kmv_request(C.Structure):
    _fields_ = [("mesh", C.c_void_p), ("precision", C.c_int), ("dt", C.c_double), ("n_steps", C.c_int64),
                ("c", C.POINTER(C.c_double)), ("eta", C.POINTER(C.c_double)), ("xs", C.POINTER(C.c_double)),
                ("n_src", C.c_int), ("f0", C.c_double), ("t0", C.c_double), ("amp", C.c_double),
                ("xr", C.POINTER(C.c_double)), ("n_rec", C.c_int), ("forward_only", C.c_int),
                ("observed", C.c_void_p), ("n_shots", C.c_int), ("absorbing", C.c_int),
                ("wavelets", C.POINTER(C.c_double))]


class kmv_result(C.Structure):
    _fields_ = [("status", C.c_int), ("J", C.c_double), ("traces", C.c_void_p),
                ("grad", C.POINTER(C.c_double)), ("n_steps", C.c_int64), ("n_rec", C.c_int64),
                ("n_dofs", C.c_int64), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("device_bytes", C.c_size_t), ("n_shots", C.c_int64)]


_lib = None
_P = C.c_void_p
_D = C.POINTER(C.c_double)


def lib():
    """Load the HIP library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2108_10946_amd.build`"
                           " (there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    sig = {
        "kmv_last_error": (C.c_char_p, []),
        "kmv_element_tables": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_int), _D, _D, _D]),
        "kmv_mesh_create": (C.c_int, [C.c_int, C.c_int, _D, C.c_int64, C.POINTER(C.c_int32), C.c_int64,
                                      C.c_int, C.POINTER(_P)]),
        "kmv_mesh_info": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int),
                                    C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
        "kmv_mesh_dof_coords": (C.c_int, [_P, _D]),
        "kmv_mesh_lumped_mass": (C.c_int, [_P, _D]),
        "kmv_mesh_boundary_mass": (C.c_int, [_P, _D]),
        "kmv_mesh_cell_dofs": (C.c_int, [_P, C.POINTER(C.c_int64)]),
        "kmv_mesh_validate": (C.c_int, [_P]),
        "kmv_mesh_patch_stats": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                           C.POINTER(C.c_int64)]),
        "kmv_mesh_destroy": (C.c_int, [_P]),
        "kmv_problem_create": (C.c_int, [_P, C.POINTER(kmv_options), C.POINTER(_P)]),
        "kmv_cfl_dt": (C.c_int, [_P, _D, _D]),
        "kmv_spectral_radius": (C.c_int, [_P, _P, C.c_int, C.c_uint64, _D, _P]),
        "kmv_set_damping": (C.c_int, [_P, _D]),
        "kmv_set_pml": (C.c_int, [_P, _D]),
        "kmv_set_absorbing_boundary": (C.c_int, [_P, C.c_int]),
        "kmv_set_sources": (C.c_int, [_P, _D, C.c_int, C.c_double, C.c_double, C.c_double]),
        "kmv_set_source_wavelet": (C.c_int, [_P, _D]),
        "kmv_set_source_wavelets": (C.c_int, [_P, _D]),
        "kmv_set_receivers": (C.c_int, [_P, _D, C.c_int]),
        "kmv_forward": (C.c_int, [_P, _P, _P, _P]),
        "kmv_forward_noalloc": (C.c_int, [_P, _P, _P, _P]),
        "kmv_misfit_gradient": (C.c_int, [_P, _P, _P, _D, _P, _P, _P]),
        "kmv_misfit_gradient_accumulate": (C.c_int, [_P, _P, _P, _D, _P, _P, _P]),
        "kmv_misfit": (C.c_int, [_P, _P, _P, _D, _P, _P]),
        "kmv_problem_status": (C.c_int, [_P, _P]),
        "kmv_adjoint": (C.c_int, [_P, _P, _P, _P, _P, _P]),
        "kmv_stiffness_apply": (C.c_int, [_P, _P, _P, _P, _P]),
        "kmv_problem_num_shots": (C.c_int, [_P, C.POINTER(C.c_int)]),
        "kmv_problem_info": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int),
                                       C.POINTER(C.c_int), C.POINTER(C.c_int64)]),
        "kmv_profile_enable": (C.c_int, [_P, C.c_int]),
        "kmv_profile_read": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_double)]),
        "kmv_problem_destroy": (C.c_int, [_P]),
        "kmv_server_create": (C.c_int, [C.c_size_t, C.c_int, C.POINTER(_P)]),
        "kmv_server_submit": (C.c_int, [_P, C.POINTER(kmv_request), C.POINTER(C.c_uint64)]),
        "kmv_server_poll": (C.c_int, [_P, C.c_uint64, C.POINTER(kmv_result)]),
        "kmv_server_wait": (C.c_int, [_P, C.c_uint64, C.c_double, C.POINTER(kmv_result)]),
        "kmv_server_release": (C.c_int, [_P, C.c_uint64]),
        "kmv_server_stats": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_size_t)]),
        "kmv_server_destroy": (C.c_int, [_P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc):
    if rc != KMV_OK:
        raise KMVError(rc, lib().kmv_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(_D)


def _tptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("device buffers must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# --------------------------------------------------------------- same-name calls
def kmv_last_error():
    return lib().kmv_last_error().decode()


def kmv_element_tables(dim, degree):
    n = C.c_int()
    _check(lib().kmv_element_tables(dim, degree, C.byref(n), None, None, None))
    nodes = np.zeros(n.value * dim)
    w = np.zeros(n.value)
    g = np.zeros(n.value * n.value * dim)
    _check(lib().kmv_element_tables(dim, degree, C.byref(n), _dptr(nodes), _dptr(w), _dptr(g)))
    return nodes.reshape(n.value, dim), w, g.reshape(n.value, n.value, dim)


def kmv_mesh_create(dim, degree, coords, cells, patch_cells=0):
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    h = _P()
    _check(lib().kmv_mesh_create(dim, degree, _dptr(coords), len(coords),
                                 cells.ctypes.data_as(C.POINTER(C.c_int32)), len(cells), patch_cells,
                                 C.byref(h)))
    return h


def kmv_mesh_info(m):
    v = [C.c_int64(), C.c_int64(), C.c_int(), C.c_int64(), C.c_int64()]
    _check(lib().kmv_mesh_info(m, *[C.byref(x) for x in v]))
    return dict(n_dofs=v[0].value, n_cells=v[1].value, n_nodes=v[2].value, n_patches=v[3].value,
                n_shared_dofs=v[4].value)


def kmv_mesh_dof_coords(m, dim):
    n = kmv_mesh_info(m)["n_dofs"]
    out = np.zeros(n * dim)
    _check(lib().kmv_mesh_dof_coords(m, _dptr(out)))
    return out.reshape(n, dim)


def kmv_mesh_lumped_mass(m):
    out = np.zeros(kmv_mesh_info(m)["n_dofs"])
    _check(lib().kmv_mesh_lumped_mass(m, _dptr(out)))
    return out


def kmv_mesh_boundary_mass(m):
    out = np.zeros(kmv_mesh_info(m)["n_dofs"])
    _check(lib().kmv_mesh_boundary_mass(m, _dptr(out)))
    return out


def kmv_mesh_cell_dofs(m):
    info = kmv_mesh_info(m)
    out = np.zeros(info["n_cells"] * info["n_nodes"], dtype=np.int64)
    _check(lib().kmv_mesh_cell_dofs(m, out.ctypes.data_as(C.POINTER(C.c_int64))))
    return out.reshape(info["n_cells"], info["n_nodes"])


def kmv_mesh_destroy(m):
    _check(lib().kmv_mesh_destroy(m))


def kmv_problem_create(m, precision, dt, n_steps, checkpoint_every=0, mem_budget=0, n_shots=1,
                       gradient_every=1):
    opt = kmv_options(precision, dt, n_steps, checkpoint_every, mem_budget, n_shots, gradient_every)
    h = _P()
    _check(lib().kmv_problem_create(m, C.byref(opt), C.byref(h)))
    return h


def kmv_problem_info(p):
    v = [C.c_int64(), C.c_int64(), C.c_int(), C.c_int(), C.c_int64()]
    _check(lib().kmv_problem_info(p, *[C.byref(x) for x in v]))
    return dict(n_dofs=v[0].value, n_steps=v[1].value, n_rec=v[2].value, precision=v[3].value,
                checkpoint_every=v[4].value)


def kmv_problem_num_shots(p):
    n = C.c_int()
    _check(lib().kmv_problem_num_shots(p, C.byref(n)))
    return n.value


def kmv_cfl_dt(m, c_host):
    c_host = np.ascontiguousarray(c_host, dtype=np.float64)
    out = C.c_double()
    _check(lib().kmv_cfl_dt(m, _dptr(c_host), C.byref(out)))
    return out.value


def kmv_mesh_validate(m):
    _check(lib().kmv_mesh_validate(m))


def kmv_mesh_patch_stats(m, adjoint=False):
    v = [C.c_int64(), C.c_int64(), C.c_int64()]
    _check(lib().kmv_mesh_patch_stats(m, 1 if adjoint else 0, *[C.byref(x) for x in v]))
    return dict(max_patch_cells=v[0].value, max_shared_refs=v[1].value, first_batch_refs=v[2].value)


def kmv_spectral_radius(p, c_dev, iters=200, seed=0, stream=None):
    out = C.c_double()
    _check(lib().kmv_spectral_radius(p, _tptr(c_dev), iters, seed, C.byref(out), _stream(stream)))
    return out.value


def kmv_set_absorbing_boundary(p, enable):
    _check(lib().kmv_set_absorbing_boundary(p, 1 if enable else 0))


def kmv_set_damping(p, eta):
    if eta is None:
        _check(lib().kmv_set_damping(p, None))
    else:
        eta = np.ascontiguousarray(eta, dtype=np.float64)
        _check(lib().kmv_set_damping(p, _dptr(eta)))


def kmv_set_pml(p, sigma, dim=2):
    """sigma: [n_dofs, dim] (sigma_x, sigma_z per DOF on triangles; sigma_x, sigma_y,
    sigma_z on tetrahedra), or None (off)."""
    if sigma is None:
        _check(lib().kmv_set_pml(p, None))
    else:
        sigma = np.ascontiguousarray(sigma, dtype=np.float64)
        if sigma.ndim != 2 or sigma.shape[1] != dim:
            raise ValueError(f"sigma must be [n_dofs, {dim}]")
        _check(lib().kmv_set_pml(p, _dptr(sigma)))


def kmv_set_sources(p, xs, f0, t0, amp=1.0):
    xs = np.ascontiguousarray(np.atleast_2d(xs), dtype=np.float64)
    _check(lib().kmv_set_sources(p, _dptr(xs), len(xs), f0, t0, amp))


def kmv_set_source_wavelet(p, w):
    w = np.ascontiguousarray(w, dtype=np.float64)
    _check(lib().kmv_set_source_wavelet(p, _dptr(w)))


def kmv_set_source_wavelets(p, w):
    w = np.ascontiguousarray(w, dtype=np.float64)
    _check(lib().kmv_set_source_wavelets(p, _dptr(w)))


def kmv_set_receivers(p, xr):
    xr = np.ascontiguousarray(np.atleast_2d(xr), dtype=np.float64)
    _check(lib().kmv_set_receivers(p, _dptr(xr), len(xr)))


def kmv_forward(p, c_dev, traces_dev, stream=None):
    _check(lib().kmv_forward(p, _tptr(c_dev), _tptr(traces_dev), _stream(stream)))


def kmv_forward_noalloc(p, c_dev, traces_dev, stream=None):
    _check(lib().kmv_forward_noalloc(p, _tptr(c_dev), _tptr(traces_dev), _stream(stream)))


def kmv_misfit_gradient(p, c_dev, observed_dev, grad_dev, traces_dev=None, stream=None):
    J = C.c_double()
    _check(lib().kmv_misfit_gradient(p, _tptr(c_dev), _tptr(observed_dev), C.byref(J), _tptr(grad_dev),
                                     _tptr(traces_dev), _stream(stream)))
    return J.value


def kmv_misfit_gradient_accumulate(p, c_dev, observed_dev, J_acc, grad_acc, traces_dev=None, stream=None):
    """Returns J_acc + J; grad_acc (device) receives grad_acc + dJ/dc."""
    J = C.c_double(J_acc)
    _check(lib().kmv_misfit_gradient_accumulate(p, _tptr(c_dev), _tptr(observed_dev), C.byref(J),
                                                _tptr(grad_acc), _tptr(traces_dev), _stream(stream)))
    return J.value


def kmv_misfit(p, c_dev, observed_dev, traces_dev=None, stream=None):
    J = C.c_double()
    _check(lib().kmv_misfit(p, _tptr(c_dev), _tptr(observed_dev), C.byref(J), _tptr(traces_dev),
                            _stream(stream)))
    return J.value


def kmv_problem_status(p, stream=None):
    _check(lib().kmv_problem_status(p, _stream(stream)))


def kmv_adjoint(p, c_dev, adj_src_dev, lambda_out_dev=None, src_trace_dev=None, stream=None):
    _check(lib().kmv_adjoint(p, _tptr(c_dev), _tptr(adj_src_dev), _tptr(lambda_out_dev),
                             _tptr(src_trace_dev), _stream(stream)))


def kmv_stiffness_apply(p, c_dev, u_dev, y_dev, stream=None):
    _check(lib().kmv_stiffness_apply(p, _tptr(c_dev), _tptr(u_dev), _tptr(y_dev), _stream(stream)))


PROFILE_VARIANTS = {0: "patch_forward", 1: "patch_adjoint", 2: "shared_forward", 3: "shared_adjoint",
                    4: "receivers"}


def kmv_profile_enable(p, every):
    _check(lib().kmv_profile_enable(p, every))


def kmv_profile_read(p, variant):
    n, t, ms = C.c_int64(), C.c_int64(), C.c_double()
    _check(lib().kmv_profile_read(p, variant, C.byref(n), C.byref(t), C.byref(ms)))
    return dict(launches=n.value, timed=t.value, mean_ms=ms.value)


def kmv_problem_destroy(p):
    _check(lib().kmv_problem_destroy(p))


# -------------------------------------------------------------------- serving
def kmv_server_create(mem_budget=0, max_slots=4):
    h = _P()
    _check(lib().kmv_server_create(mem_budget, max_slots, C.byref(h)))
    return h


def kmv_server_submit(s, mesh, precision, dt, n_steps, c, xs, xr, f0, t0, amp=1.0, eta=None,
                      observed=None, forward_only=False, absorbing=False, wavelets=None):
    """Queue one request.  xs is [n_src, dim] for one shot or [n_shots, n_src, dim]
    for several (observed then [n_shots, n_steps, n_rec]).  wavelets: None (the
    Ricker wavelet of f0, t0, amp for every shot) or [n_shots, n_steps], one per
    shot.  Host inputs are copied before this returns."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    if mesh is not None:  # the library copies n_dofs values from c and eta
        n_dofs = kmv_mesh_info(mesh)["n_dofs"]
        if c.size != n_dofs:
            raise ValueError(f"c must hold the mesh's {n_dofs} DOF values, got {c.size}")
        if eta is not None and np.size(eta) != n_dofs:
            raise ValueError(f"eta must hold the mesh's {n_dofs} DOF values, got {np.size(eta)}")
    xs = np.asarray(xs, dtype=np.float64)
    n_shots = xs.shape[0] if xs.ndim == 3 else 1
    xs = np.ascontiguousarray(xs.reshape(-1, xs.shape[-1]) if xs.ndim == 3 else np.atleast_2d(xs))
    xr = np.ascontiguousarray(np.atleast_2d(xr), dtype=np.float64)
    eta = None if eta is None else np.ascontiguousarray(eta, dtype=np.float64)
    obs = None
    if not forward_only:
        obs = np.ascontiguousarray(observed, dtype=np.float64 if precision == KMV_FP64 else np.float32)
        if obs.size != n_shots * n_steps * len(xr):
            raise ValueError("observed must hold n_shots * n_steps * n_rec values")
    if wavelets is not None:
        wavelets = np.ascontiguousarray(wavelets, dtype=np.float64)
        if wavelets.size != n_shots * n_steps:
            raise ValueError("wavelets must hold n_shots * n_steps values")
    req = kmv_request(mesh, precision, dt, n_steps, _dptr(c), None if eta is None else _dptr(eta), _dptr(xs),
                      len(xs), f0, t0, amp, _dptr(xr), len(xr), 1 if forward_only else 0,
                      None if obs is None else obs.ctypes.data_as(C.c_void_p), n_shots, 1 if absorbing else 0,
                      None if wavelets is None else _dptr(wavelets))
    t = C.c_uint64()
    _check(lib().kmv_server_submit(s, C.byref(req), C.byref(t)))
    return t.value


def _result_dict(r, precision_hint=None):
    out = dict(status=r.status, J=r.J, n_steps=r.n_steps, n_rec=r.n_rec, n_dofs=r.n_dofs, n_shots=r.n_shots,
               t_submit=r.t_submit, t_admit=r.t_admit, t_done=r.t_done, device_bytes=r.device_bytes,
               traces=None, grad=None)
    if r.status == KMV_OK:
        n = r.n_shots * r.n_steps * r.n_rec
        shape = (r.n_steps, r.n_rec) if r.n_shots == 1 else (r.n_shots, r.n_steps, r.n_rec)
        if r.traces:
            ct = C.c_double if precision_hint == KMV_FP64 else C.c_float
            buf = (ct * n).from_address(r.traces)
            out["traces"] = np.array(np.frombuffer(buf, dtype=np.float64 if ct is C.c_double else np.float32),
                                     copy=True).reshape(shape)
        if r.grad:
            out["grad"] = np.array(np.ctypeslib.as_array(r.grad, shape=(r.n_dofs,)), copy=True)
    else:
        out["error"] = kmv_last_error()
    return out


def kmv_server_poll(s, ticket, precision):
    """None while pending, else the result (copied out of the library's buffers)."""
    r = kmv_result()
    rc = lib().kmv_server_poll(s, ticket, C.byref(r))
    if rc == KMV_EBUSY:
        return None
    _check(rc)
    return _result_dict(r, precision)


def kmv_server_wait(s, ticket, precision, timeout_s=-1.0):
    r = kmv_result()
    rc = lib().kmv_server_wait(s, ticket, timeout_s, C.byref(r))
    if rc == KMV_EBUSY:
        return None
    _check(rc)
    return _result_dict(r, precision)


def kmv_server_release(s, ticket):
    _check(lib().kmv_server_release(s, ticket))


def kmv_server_stats(s):
    v = [C.c_int(), C.c_int(), C.c_size_t()]
    _check(lib().kmv_server_stats(s, *[C.byref(x) for x in v]))
    return dict(running=v[0].value, queued=v[1].value, bytes_in_use=v[2].value)


def kmv_server_destroy(s):
    _check(lib().kmv_server_destroy(s))
