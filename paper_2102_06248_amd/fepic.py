"""ctypes binding of libfepic (include/fepic.h): argument marshalling only.

Every function here has the name of the C entry point it calls and converts numpy arrays
to pointers and back; all of the method's work happens in the library's HIP kernels.
The library must have been built (``python -m paper_2102_06248_amd.build``); importing
this module without it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfepic.so")

ABI_VERSION = 8   # include/fepic.h FEPIC_ABI_VERSION: layouts of the structs below
FEPIC_OK = 0
FEPIC_FP32_PUSH_FP64_ACC, FEPIC_ALL_FP64 = 0, 1
FEPIC_WS_PREV, FEPIC_WS_EXTRAP1, FEPIC_WS_EXTRAP2, FEPIC_WS_MLP, FEPIC_WS_MLP_DIRECT = 0, 1, 2, 3, 4
FEPIC_PC_JACOBI, FEPIC_PC_AUX = 0, 1
FEPIC_WALK_AUTO, FEPIC_WALK_QUEUE, FEPIC_WALK_FUSED = 0, 1, 2
FEPIC_SORT_AUTO = -1
FEPIC_SOLVE_FP64, FEPIC_SOLVE_MIXED = 0, 1
FEPIC_PUSHER_BORIS, FEPIC_PUSHER_AB = 0, 1
FEPIC_FIELD_WAVE, FEPIC_FIELD_NM_MFEM, FEPIC_FIELD_BD_MFEM = 0, 1, 2
FEPIC_E_CG_NOT_CONVERGED = -6
FEPIC_E_CROSSING_CAP = -7
FEPIC_MLP_N_PARAMS = 4545
FEPIC_MLP_NOALLOC_MAX_ROWS = 65536   # include/fepic.h

ERROR_NAMES = {-1: "FEPIC_E_ARG", -2: "FEPIC_E_MESH", -3: "FEPIC_E_STATE", -4: "FEPIC_E_OOM", -5: "FEPIC_E_HIP",
               -6: "FEPIC_E_CG_NOT_CONVERGED", -7: "FEPIC_E_CROSSING_CAP", -8: "FEPIC_E_IO", -9: "FEPIC_E_NO_DEVICE"}


class fepic_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("precision", ctypes.c_int), ("cg_tol", ctypes.c_double),
                ("cg_max_iters", ctypes.c_int), ("cg_check_every", ctypes.c_int), ("sort_period", ctypes.c_int),
                ("crossing_cap", ctypes.c_int), ("warm_start", ctypes.c_int), ("diagnostics", ctypes.c_int),
                ("timing", ctypes.c_int), ("preconditioner", ctypes.c_int), ("aux_far_levels", ctypes.c_int),
                ("walk", ctypes.c_int), ("solve_precision", ctypes.c_int), ("mixed_inner_tol", ctypes.c_double),
                ("pusher", ctypes.c_int), ("ab_order", ctypes.c_int), ("field_solver", ctypes.c_int),
                ("deterministic", ctypes.c_int)]


class fepic_step_stats(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("t", ctypes.c_double), ("cg_iters", ctypes.c_int),
                ("cg_rel_resid", ctypes.c_double), ("cg_rel_resid0", ctypes.c_double),
                ("cont_resid_rel", ctypes.c_double), ("gauss_resid_rel", ctypes.c_double),
                ("gauss_drift_check_rel", ctypes.c_double), ("divb_max", ctypes.c_double),
                ("field_energy", ctypes.c_double), ("n_particles", ctypes.c_int64), ("n_absorbed", ctypes.c_int64),
                ("n_crossings", ctypes.c_int64), ("max_crossings", ctypes.c_int), ("n_cap_exceeded", ctypes.c_int),
                ("ms_sort", ctypes.c_float), ("ms_stage", ctypes.c_float), ("ms_particles", ctypes.c_float),
                ("ms_rhs", ctypes.c_float), ("ms_warm", ctypes.c_float), ("ms_cg", ctypes.c_float),
                ("ms_faraday", ctypes.c_float), ("ms_diag", ctypes.c_float),
                ("magnetic_energy", ctypes.c_double), ("kinetic_energy", ctypes.c_double),
                ("pc_far_levels", ctypes.c_int), ("cg_passes", ctypes.c_int), ("n_injected", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class fepic_injector(ctypes.Structure):
    _fields_ = [("center", ctypes.c_double * 3), ("normal", ctypes.c_double * 3), ("radius", ctypes.c_double),
                ("kinetic_eV", ctypes.c_double), ("thermal_eV", ctypes.c_double), ("per_step", ctypes.c_int64),
                ("seed", ctypes.c_uint64)]


class fepic_train_opts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int64), ("lr", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("val_fraction", ctypes.c_double)]


class fepic_train_stats(ctypes.Structure):
    _fields_ = [("train_loss", ctypes.c_double), ("val_loss", ctypes.c_double), ("n_train_rows", ctypes.c_int64),
                ("n_val_rows", ctypes.c_int64), ("n_steps", ctypes.c_int64), ("ms_total", ctypes.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_PI64 = ctypes.POINTER(ctypes.c_int64)
_D = ctypes.c_double
_INT = ctypes.c_int

# name -> argtypes (every entry point returns int unless listed in _RESTYPES)
_SIGS = {
    "fepic_abi_version": [],
    "fepic_default_options": [ctypes.POINTER(fepic_options)],
    "fepic_error_string": [_INT],
    "fepic_last_error": [_P],
    "fepic_create": [ctypes.POINTER(fepic_options), ctypes.POINTER(_P)],
    "fepic_destroy": [_P],
    "fepic_set_stream": [_P, _P],
    "fepic_set_allocator": [_P, _P, _P, _P],
    "fepic_upload_mesh": [_P, _I64, _P, _I64, _P],
    "fepic_get_topology_sizes": [_P, _PI64, _PI64, _PI64, _PI64, _PI64],
    "fepic_get_topology": [_P, _P, _P, _P, _P, _P, _P],
    "fepic_get_matrix": [_P, _INT, _I64, _PI64, _P, _P, _P],
    "fepic_set_fields": [_P, _P, _P, _P],
    "fepic_set_uniform_B": [_P, _P],
    "fepic_init_electrostatic": [_P, _D, ctypes.POINTER(_INT)],
    "fepic_add_species": [_P, _D, _D, _D, ctypes.POINTER(_INT)],
    "fepic_upload_particles": [_P, _INT, _I64, _P, _P, _P, _PI64],
    "fepic_set_injector": [_P, _INT, ctypes.POINTER(fepic_injector)],
    "fepic_inject_particles": [_P, _INT, _I64, _P, _P, _P],
    "fepic_inject_particles_device": [_P, _INT, _I64, _P, _P, _P],
    "fepic_upload_particles_device": [_P, _INT, _I64, _P, _P, _P, _PI64],
    "fepic_num_particles": [_P, _INT, _PI64],
    "fepic_get_particles": [_P, _INT, _I64, _PI64, _P, _P, _P, _P, _P],
    "fepic_step": [_P, _D, _D, _D, ctypes.POINTER(fepic_step_stats)],
    "fepic_push_particles": [_P, _D, ctypes.POINTER(fepic_step_stats)],
    "fepic_get_fields": [_P, _P, _P, _P],
    "fepic_get_current": [_P, _P, _P],
    "fepic_get_rho": [_P, _P],
    "fepic_diagnostics": [_P, ctypes.POINTER(fepic_step_stats)],
    "fepic_kernel_timing": [_P, ctypes.c_char_p, _INT],
    "fepic_kernel_time": [_P, ctypes.c_char_p, ctypes.POINTER(_D), _PI64],
    "fepic_ws_record": [_P, _INT, _I64],
    "fepic_ws_num_snapshots": [_P, _PI64],
    "fepic_ws_train": [_P, ctypes.POINTER(fepic_train_opts), ctypes.POINTER(fepic_train_stats)],
    "fepic_ws_get_weights": [_P, _P, _I64, _PI64],
    "fepic_ws_set_weights": [_P, _P, _I64],
    "fepic_set_warm_start": [_P, _INT],
    "fepic_set_preconditioner": [_P, _INT],
    "fepic_set_solve_precision": [_P, _INT],
    "fepic_set_pusher": [_P, _INT, _INT],
    "fepic_set_field_solver": [_P, _INT],
    "fepic_set_absorbing_faces": [_P, _I64, _P],
    "fepic_mlp_forward": [_P, _I64, _P, _P],
    "fepic_mlp_grad": [_P, _I64, _P, _P, _P, ctypes.POINTER(_D)],
    "fepic_mlp_grad_noalloc": [_P, _I64, _P, _P, _P, _P],
    "fepic_mlp_adam_step": [_P, _P, _D, _D, _D, _D],
    "fepic_keep_warm_start": [_P, _INT],
    "fepic_get_warm_start": [_P, _P],
    "fepic_save": [_P, ctypes.c_char_p],
    "fepic_load": [_P, ctypes.c_char_p],
}
_RESTYPES = {"fepic_default_options": None, "fepic_error_string": ctypes.c_char_p,
             "fepic_last_error": ctypes.c_char_p}

_lib = None


def lib():
    """The loaded libfepic (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfepic.so is not built; run `python -m paper_2102_06248_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _RESTYPES.get(name, ctypes.c_int)
        if L.fepic_abi_version() != ABI_VERSION:
            raise RuntimeError(f"libfepic.so has ABI version {L.fepic_abi_version()}, this binding expects "
                               f"{ABI_VERSION}; rebuild with `python -m paper_2102_06248_amd.build`")
        _lib = L
    return _lib


class FepicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def fepic_error_string(code):
    return lib().fepic_error_string(code).decode()


def fepic_last_error(ctx):
    return lib().fepic_last_error(ctx).decode()


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(ctx, rc):
    if rc != FEPIC_OK:
        msg = lib().fepic_last_error(ctx).decode() if ctx else lib().fepic_error_string(rc).decode()
        raise FepicError(rc, msg)


def _arr(a, dtype, shape=None):
    out = np.ascontiguousarray(a, dtype=dtype)
    if shape is not None:
        out = out.reshape(shape)
    return out


# ------------------------------------------------------------------ entry points, same names

def fepic_abi_version():
    return lib().fepic_abi_version()


def fepic_default_options():
    o = fepic_options()
    lib().fepic_default_options(ctypes.byref(o))
    return o


def fepic_create(opts=None, **kw):
    o = opts if opts is not None else fepic_default_options()
    for k, v in kw.items():
        setattr(o, k, v)
    ctx = ctypes.c_void_p()
    _check(None, lib().fepic_create(ctypes.byref(o), ctypes.byref(ctx)))
    return ctx


def fepic_destroy(ctx):
    _check(None, lib().fepic_destroy(ctx))


def fepic_set_stream(ctx, stream_handle):
    _check(ctx, lib().fepic_set_stream(ctx, ctypes.c_void_p(stream_handle)))


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def fepic_set_allocator(ctx, alloc_fn, free_fn):
    """alloc_fn(nbytes) -> device address (int) or None; free_fn(address).  Returns the
    ctypes callbacks, which the caller must keep alive as long as the context."""
    def _a(n, user):
        p = alloc_fn(n)
        return p if p else None

    def _f(p, user):
        free_fn(p)

    cbs = (ALLOC_FN(_a), FREE_FN(_f))
    _check(ctx, lib().fepic_set_allocator(ctx, ctypes.cast(cbs[0], ctypes.c_void_p),
                                          ctypes.cast(cbs[1], ctypes.c_void_p), None))
    return cbs


def torch_allocator(device=0):
    """(alloc_fn, free_fn) routing the library's device memory through torch's caching
    allocator on the given device."""
    import torch

    def alloc_fn(n):
        try:
            return torch.cuda.caching_allocator_alloc(n, device)
        except RuntimeError:
            return None

    def free_fn(p):
        torch.cuda.caching_allocator_delete(p)

    return alloc_fn, free_fn


def fepic_upload_mesh(ctx, xyz, tets):
    xyz = _arr(xyz, np.float64, (-1, 3))
    tets = _arr(tets, np.int32, (-1, 4))
    _check(ctx, lib().fepic_upload_mesh(ctx, len(xyz), _ptr(xyz), len(tets), _ptr(tets)))


def fepic_get_topology_sizes(ctx):
    v = [ctypes.c_int64() for _ in range(5)]
    _check(ctx, lib().fepic_get_topology_sizes(ctx, *[ctypes.byref(x) for x in v]))
    return dict(zip(["n_edges", "n_faces", "n_int_edges", "n_int_nodes", "euler"], [x.value for x in v]))


def fepic_get_topology(ctx, n_tets):
    s = fepic_get_topology_sizes(ctx)
    out = {"tets": np.zeros((n_tets, 4), np.int32), "edges": np.zeros((s["n_edges"], 2), np.int32),
           "faces": np.zeros((s["n_faces"], 3), np.int32), "tet_edges": np.zeros((n_tets, 6), np.int32),
           "tet_faces": np.zeros((n_tets, 4), np.int32), "nbr": np.zeros((n_tets, 4), np.int32)}
    _check(ctx, lib().fepic_get_topology(ctx, *[_ptr(out[k]) for k in
                                                ("tets", "edges", "faces", "tet_edges", "tet_faces", "nbr")]))
    return out


def fepic_get_matrix(ctx, which):
    n = ctypes.c_int64()
    _check(ctx, lib().fepic_get_matrix(ctx, which, 0, ctypes.byref(n), None, None, None))
    r = np.zeros(n.value, np.int64)
    c = np.zeros(n.value, np.int64)
    v = np.zeros(n.value, np.float64)
    _check(ctx, lib().fepic_get_matrix(ctx, which, n.value, ctypes.byref(n), _ptr(r), _ptr(c), _ptr(v)))
    return r, c, v


def fepic_get_matrix_nnz(ctx, which):
    """Stored entries of matrix `which` (0 = M, 1 = S, 2 = K) over the unknown edges."""
    n = ctypes.c_int64()
    _check(ctx, lib().fepic_get_matrix(ctx, which, 0, ctypes.byref(n), None, None, None))
    return n.value


def fepic_set_fields(ctx, e=None, e_prev=None, b=None):
    e = None if e is None else _arr(e, np.float64)
    e_prev = None if e_prev is None else _arr(e_prev, np.float64)
    b = None if b is None else _arr(b, np.float64)
    _check(ctx, lib().fepic_set_fields(ctx, _ptr(e), _ptr(e_prev), _ptr(b)))


def fepic_set_uniform_B(ctx, B0):
    B0 = _arr(B0, np.float64)
    _check(ctx, lib().fepic_set_uniform_B(ctx, _ptr(B0)))


def fepic_init_electrostatic(ctx, tol=1e-14):
    it = ctypes.c_int()
    _check(ctx, lib().fepic_init_electrostatic(ctx, tol, ctypes.byref(it)))
    return it.value


def fepic_add_species(ctx, q, m, w):
    s = ctypes.c_int()
    _check(ctx, lib().fepic_add_species(ctx, q, m, w, ctypes.byref(s)))
    return s.value


def fepic_upload_particles(ctx, species, x, u, ids=None):
    x = _arr(x, np.float64, (-1, 3))
    u = _arr(u, np.float64, (-1, 3))
    ids = None if ids is None else _arr(ids, np.int64)
    rej = ctypes.c_int64()
    _check(ctx, lib().fepic_upload_particles(ctx, species, len(x), _ptr(ids), _ptr(x), _ptr(u), ctypes.byref(rej)))
    return rej.value


def fepic_inject_particles(ctx, species, x, u, ids=None):
    x = _arr(x, np.float64, (-1, 3))
    u = _arr(u, np.float64, (-1, 3))
    ids = None if ids is None else _arr(ids, np.int64)
    _check(ctx, lib().fepic_inject_particles(ctx, species, len(x), _ptr(ids), _ptr(x), _ptr(u)))


def fepic_upload_particles_device(ctx, species, n, x_ptr, u_ptr, id_ptr=None):
    """Device addresses as for fepic_inject_particles_device; returns the rejected count."""
    rej = ctypes.c_int64()
    _check(ctx, lib().fepic_upload_particles_device(ctx, species, n, id_ptr, x_ptr, u_ptr, ctypes.byref(rej)))
    return rej.value


def fepic_inject_particles_device(ctx, species, n, x_ptr, u_ptr, id_ptr=None):
    """x_ptr, u_ptr: device addresses of [n][3] float64 arrays (e.g. tensor.data_ptr());
    id_ptr: device address of [n] int64 ids, or None."""
    _check(ctx, lib().fepic_inject_particles_device(ctx, species, n, id_ptr, x_ptr, u_ptr))


def fepic_set_injector(ctx, species, center=None, normal=None, radius=None, kinetic_eV=0.0, thermal_eV=0.0,
                       per_step=0, seed=0, off=False):
    """Seeded disk source of a species (off=True removes it)."""
    if off:
        _check(ctx, lib().fepic_set_injector(ctx, int(species), None))
        return
    spec = fepic_injector((ctypes.c_double * 3)(*center), (ctypes.c_double * 3)(*normal), float(radius),
                          float(kinetic_eV), float(thermal_eV), int(per_step), int(seed))
    _check(ctx, lib().fepic_set_injector(ctx, int(species), ctypes.byref(spec)))


def fepic_num_particles(ctx, species):
    n = ctypes.c_int64()
    _check(ctx, lib().fepic_num_particles(ctx, species, ctypes.byref(n)))
    return n.value


def fepic_get_particles(ctx, species, fields=("id", "x", "u", "tet", "lam")):
    """Live particles of a species; only the named arrays are copied out (the others are
    passed as NULL)."""
    cap = fepic_num_particles(ctx, species)
    shapes = {"id": ((cap,), np.int64), "x": ((cap, 3), np.float64), "u": ((cap, 3), np.float64),
              "tet": ((cap,), np.int32), "lam": ((cap, 4), np.float64)}
    out = {k: np.zeros(*shapes[k]) for k in fields}
    n = ctypes.c_int64()
    ptrs = [_ptr(out[k]) if k in out else None for k in ("id", "x", "u", "tet", "lam")]
    _check(ctx, lib().fepic_get_particles(ctx, species, cap, ctypes.byref(n), *ptrs))
    return {k: v[:n.value] for k, v in out.items()}


def fepic_step(ctx, dt, beta=0.25, gamma=0.5, check=True):
    st = fepic_step_stats()
    rc = lib().fepic_step(ctx, dt, beta, gamma, ctypes.byref(st))
    if check:
        _check(ctx, rc)
        return st
    return rc, st


def fepic_push_particles(ctx, dt):
    st = fepic_step_stats()
    _check(ctx, lib().fepic_push_particles(ctx, dt, ctypes.byref(st)))
    return st


def fepic_get_fields(ctx):
    s = fepic_get_topology_sizes(ctx)
    e = np.zeros(s["n_edges"])
    ep = np.zeros(s["n_edges"])
    b = np.zeros(s["n_faces"])
    _check(ctx, lib().fepic_get_fields(ctx, _ptr(e), _ptr(ep), _ptr(b)))
    return e, ep, b


def fepic_get_current(ctx):
    s = fepic_get_topology_sizes(ctx)
    dg = np.zeros(s["n_edges"])
    G = np.zeros(s["n_edges"])
    _check(ctx, lib().fepic_get_current(ctx, _ptr(dg), _ptr(G)))
    return dg, G


def fepic_get_rho(ctx, n_nodes):
    rho = np.zeros(n_nodes)
    _check(ctx, lib().fepic_get_rho(ctx, _ptr(rho)))
    return rho


def fepic_keep_warm_start(ctx, on=True):
    _check(ctx, lib().fepic_keep_warm_start(ctx, int(bool(on))))


def fepic_get_warm_start(ctx):
    x0 = np.zeros(fepic_get_topology_sizes(ctx)["n_edges"])
    _check(ctx, lib().fepic_get_warm_start(ctx, _ptr(x0)))
    return x0


def fepic_mlp_adam_step(ctx, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    g = _arr(grad, np.float32)
    assert len(g) == FEPIC_MLP_N_PARAMS
    _check(ctx, lib().fepic_mlp_adam_step(ctx, _ptr(g), lr, beta1, beta2, eps))


def fepic_diagnostics(ctx):
    st = fepic_step_stats()
    _check(ctx, lib().fepic_diagnostics(ctx, ctypes.byref(st)))
    return st


def fepic_kernel_timing(ctx, family, enable):
    _check(ctx, lib().fepic_kernel_timing(ctx, family.encode(), int(enable)))


def fepic_kernel_time(ctx, family):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(ctx, lib().fepic_kernel_time(ctx, family.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def fepic_ws_record(ctx, on, max_snapshots=0):
    _check(ctx, lib().fepic_ws_record(ctx, int(on), int(max_snapshots)))


def fepic_ws_num_snapshots(ctx):
    n = ctypes.c_int64()
    _check(ctx, lib().fepic_ws_num_snapshots(ctx, ctypes.byref(n)))
    return n.value


def fepic_ws_train(ctx, epochs=4, batch=65536, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0, val_fraction=0.2):
    o = fepic_train_opts(epochs, batch, lr, beta1, beta2, eps, seed, val_fraction)
    st = fepic_train_stats()
    _check(ctx, lib().fepic_ws_train(ctx, ctypes.byref(o), ctypes.byref(st)))
    return st


def fepic_ws_get_weights(ctx):
    w = np.zeros(FEPIC_MLP_N_PARAMS, np.float32)
    n = ctypes.c_int64()
    _check(ctx, lib().fepic_ws_get_weights(ctx, _ptr(w), len(w), ctypes.byref(n)))
    return w[:n.value]


def fepic_ws_set_weights(ctx, w):
    w = _arr(w, np.float32)
    _check(ctx, lib().fepic_ws_set_weights(ctx, _ptr(w), len(w)))


def fepic_set_warm_start(ctx, mode):
    _check(ctx, lib().fepic_set_warm_start(ctx, int(mode)))


def fepic_set_preconditioner(ctx, pc):
    _check(ctx, lib().fepic_set_preconditioner(ctx, int(pc)))


def fepic_set_solve_precision(ctx, solve_precision):
    _check(ctx, lib().fepic_set_solve_precision(ctx, int(solve_precision)))


def fepic_set_field_solver(ctx, solver):
    _check(ctx, lib().fepic_set_field_solver(ctx, int(solver)))


def fepic_set_absorbing_faces(ctx, faces=None):
    """Absorbing wall faces (canonical ids); None = every wall face."""
    if faces is None:
        _check(ctx, lib().fepic_set_absorbing_faces(ctx, 0, None))
        return
    f = np.ascontiguousarray(faces, dtype=np.int32)
    _check(ctx, lib().fepic_set_absorbing_faces(ctx, len(f), _ptr(f)))


def fepic_set_pusher(ctx, pusher, ab_order=4):
    _check(ctx, lib().fepic_set_pusher(ctx, int(pusher), int(ab_order)))


def fepic_mlp_forward(ctx, X):
    X = _arr(X, np.float32, (-1, 4))
    y = np.zeros(len(X), np.float32)
    _check(ctx, lib().fepic_mlp_forward(ctx, len(X), _ptr(X), _ptr(y)))
    return y


def fepic_mlp_grad(ctx, X, t):
    X = _arr(X, np.float32, (-1, 4))
    t = _arr(t, np.float32)
    g = np.zeros(FEPIC_MLP_N_PARAMS, np.float32)
    loss = ctypes.c_double()
    _check(ctx, lib().fepic_mlp_grad(ctx, len(X), _ptr(X), _ptr(t), _ptr(g), ctypes.byref(loss)))
    return loss.value, g


def fepic_mlp_grad_noalloc(ctx, n, X_dev, t_dev, grad_dev, loss_dev):
    """Device pointers (ints, e.g. torch tensors' data_ptr()); enqueued on the context's
    stream, nothing allocated, no synchronization."""
    _check(ctx, lib().fepic_mlp_grad_noalloc(ctx, n, X_dev, t_dev, grad_dev, loss_dev))


def fepic_save(ctx, path):
    _check(ctx, lib().fepic_save(ctx, os.fsencode(path)))


def fepic_load(ctx, path):
    _check(ctx, lib().fepic_load(ctx, os.fsencode(path)))


# ------------------------------------------------------------------ convenience wrapper

class Simulation:
    """Owns one context; thin sugar over the functions above."""

    def __init__(self, xyz, tets, allocator=None, **opts):
        """allocator: None (hipMalloc) or "torch" (torch's caching allocator)."""
        self.ctx = fepic_create(**opts)
        self.n_nodes = len(xyz)
        self.n_tets = len(tets)
        self._alloc_cbs = None
        try:
            if allocator == "torch":
                self._alloc_cbs = fepic_set_allocator(self.ctx, *torch_allocator(opts.get("device", 0)))
            elif allocator is not None:
                raise ValueError(f"unknown allocator {allocator!r}")
            fepic_upload_mesh(self.ctx, xyz, tets)
        except Exception:
            self.close()
            raise
        self.sizes = fepic_get_topology_sizes(self.ctx)

    def close(self):
        if self.ctx is not None:
            fepic_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
