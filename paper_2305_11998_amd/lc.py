"""Python binding of the ``liblc`` C ABI (argument marshalling only).

Every function here has the name of the C entry point it calls and does no
arithmetic of the method: it checks tensor devices, dtypes and sizes (so the
kernels never see a buffer smaller than they assume), passes raw device
pointers and the current HIP stream, and turns non-OK status codes into
exceptions.  Device memory comes from PyTorch.  If the HIP library has not
been built this module raises at import: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
_lib = C.CDLL(LIB_PATH)

LC_OK, LC_ERR_ARG, LC_ERR_ALLOC, LC_ERR_HIP, LC_ERR_STATE, LC_ERR_UNSUPPORTED = range(6)
LC_RAYS_UNIFORM, LC_RAYS_TUBES = 0, 1
LC_F64, LC_F32 = 0, 1
_STATUS = {1: "LC_ERR_ARG", 2: "LC_ERR_ALLOC", 3: "LC_ERR_HIP", 4: "LC_ERR_STATE", 5: "LC_ERR_UNSUPPORTED"}


class LcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class lc_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("lx", C.c_double), ("ly", C.c_double)]


class lc_quad(C.Structure):
    _fields_ = [("n_az", C.c_int32), ("n_pol", C.c_int32), ("phi", C.POINTER(C.c_double)),
                ("mu", C.POINTER(C.c_double)), ("omega", C.POINTER(C.c_double))]


class lc_rays_info_t(C.Structure):
    _fields_ = [("n_rays", C.c_int64), ("n_segments", C.c_int64), ("n_pairs", C.c_int32),
                ("n_az", C.c_int32), ("n_pol", C.c_int32), ("n_cells", C.c_int32),
                ("n_faces", C.c_int32), ("max_seg_per_ray", C.c_int32), ("mode", C.c_int32),
                ("h_moc", C.c_double)]


class lc_tuning_t(C.Structure):
    _fields_ = [("sweep_unroll", C.c_int32), ("moments_entries", C.c_int32)]


class lc_problem_t(C.Structure):
    _fields_ = [("plan", C.c_void_p), ("kappa", C.c_void_p), ("planck", C.c_void_p),
                ("material_stride", C.c_int64), ("c_dt", C.c_double), ("state_a", C.c_void_p),
                ("state_b", C.c_void_p), ("I_in", C.c_void_p), ("I_exit", C.c_void_p),
                ("E", C.c_void_p), ("F", C.c_void_p), ("f", C.c_void_p), ("bnd", C.c_void_p)]


_vp, _i32, _i64, _d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
_SIGS = {
    "lc_version": ([], C.c_int32),
    "lc_last_error": ([], C.c_char_p),
    "lc_build_rays": ([C.POINTER(lc_grid), C.POINTER(lc_quad), _d, _i32, _vp, C.POINTER(_vp)], C.c_int),
    "lc_rays_free": ([_vp], C.c_int),
    "lc_rays_info": ([_vp, C.POINTER(lc_rays_info_t)], C.c_int),
    "lc_rays_export": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "lc_plan_create": ([_vp, _i32, _i32, C.POINTER(_vp)], C.c_int),
    "lc_plan_free": ([_vp], C.c_int),
    "lc_state_bytes": ([_vp], C.c_size_t),
    "lc_state_fill": ([_vp, _vp, _vp, _vp], C.c_int),
    "lc_state_export": ([_vp, _vp, _vp, _vp], C.c_int),
    "lc_state_import": ([_vp, _vp, _vp, _vp], C.c_int),
    "lc_sweep": ([_vp, _vp, _vp, _d, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "lc_sweep_noalloc": ([_vp, _vp, _vp, _d, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "lc_set_alloc_limit": ([C.c_uint64], C.c_int),
    "lc_set_validation": ([_i32], C.c_int),
    "lc_loqd_create": ([_i32, _i32, _d, _d, _i32, C.POINTER(_vp)], C.c_int),
    "lc_loqd_free": ([_vp], C.c_int),
    "lc_loqd_set_warm_start": ([_vp, _i32], C.c_int),
    "lc_loqd_set_solver": ([_vp, _i32], C.c_int),
    "lc_mlqd_create": ([_vp, _vp, _vp, _d, _d, _d, C.POINTER(_vp)], C.c_int),
    "lc_mlqd_free": ([_vp], C.c_int),
    "lc_mlqd_set_acceleration": ([_vp, _i32], C.c_int),
    "lc_mlqd_material": ([_vp, _vp, _vp, _vp, _vp], C.c_int),
    "lc_mlqd_step": ([_vp, _d] + [_vp] * 11 + [_d, _i32, _i32, _vp, _vp, _vp, _vp], C.c_int),
    "lc_loqd_solve_general": ([_vp, _d, _d, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _d, _i32, _vp,
                               _vp, _vp], C.c_int),
    "lc_loqd_grey_coefficients": ([_vp, _d, _d] + [_vp] * 21, C.c_int),
    "lc_loqd_grey_meb": ([_vp, _d, _d] + [_vp] * 10 + [_d, _d] + [_vp] * 4 + [_d, _i32, _d, _i32, _vp, _vp, _vp, _vp],
                         C.c_int),
    "lc_loqd_solve": ([_vp, _d, _d, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _d, _i32, _vp, _vp, _vp],
                      C.c_int),
    "lc_moments": ([_vp, _vp, _vp, _vp, _d, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "lc_step": ([_vp, _i32, _vp, _vp, _i64, _d, _d, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "lc_grey_closures": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "lc_grey_closures_dims": ([_i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "lc_plan_enable_faces": ([_vp, _vp], C.c_int),
    "lc_sweep_points": ([_vp, _vp, _vp, _d, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "lc_face_moments": ([_vp, _vp, _vp, _d, _vp, _vp, _vp, _vp], C.c_int),
    "lc_plan_set_tuning": ([_vp, C.POINTER(lc_tuning_t)], C.c_int),
    "lc_plan_get_tuning": ([_vp, C.POINTER(lc_tuning_t)], C.c_int),
    "lc_plan_set_split": ([_vp, _i32], C.c_int),
    "lc_plan_set_moment_split": ([_vp, _i32], C.c_int),
    "lc_plan_get_moment_split": ([_vp, _vp], C.c_int),
    "lc_plan_set_sweep_residency": ([_vp, _i32], C.c_int),
    "lc_plan_profile": ([_vp, _i32], C.c_int),
    "lc_plan_profile_read": ([_vp, _vp], C.c_int),
    "lc_batch_create": ([_i32, C.POINTER(lc_problem_t), C.POINTER(_vp)], C.c_int),
    "lc_batch_step": ([_vp, _i32, _d, _vp], C.c_int),
    "lc_batch_free": ([_vp], C.c_int),
    "lc_batch_profile": ([_vp, _i32], C.c_int),
    "lc_batch_profile_read": ([_vp, _vp], C.c_int),
}
EXPORTED = tuple(_SIGS)
for _name, (_args, _res) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res


def _check(status):
    if status != LC_OK:
        raise LcError(status, _lib.lc_last_error().decode(errors="replace"))


def lc_version() -> int:
    return _lib.lc_version()


def _stream(stream):
    import torch
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dev(t, n, dtype_name="float64", name="tensor", optional=False):
    """Raw device pointer of a contiguous CUDA tensor holding >= n elements."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a device tensor")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise TypeError(f"{name} must be {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < n:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {n}")
    return C.c_void_p(t.data_ptr())


def _bytes(t, nbytes, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous device tensor")
    if t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{name} holds {t.numel() * t.element_size()} bytes, needs {nbytes}")
    return C.c_void_p(t.data_ptr())


class Rays:
    """Owning wrapper of an ``lc_rays_t`` handle."""

    def __init__(self, handle, nx, ny, n_az, n_pol):
        self.handle = handle
        info = lc_rays_info_t()
        _check(_lib.lc_rays_info(handle, C.byref(info)))
        self.info = info
        self.nx, self.ny, self.n_az, self.n_pol = nx, ny, n_az, n_pol
        self.n_rays = info.n_rays
        self.n_segments = info.n_segments
        self.n_pairs = info.n_pairs
        self.cells = info.n_cells
        self.nb = info.n_faces
        self.M = n_az * n_pol

    def free(self):
        if self.handle:
            _check(_lib.lc_rays_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def lc_build_rays(nx, ny, lx, ly, phi, mu, omega, h_moc, mode=LC_RAYS_UNIFORM, stream=None) -> Rays:
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    if omega.size != phi.size * mu.size:
        raise ValueError("omega must have n_az * n_pol entries")
    g = lc_grid(int(nx), int(ny), float(lx), float(ly))
    dp = C.POINTER(C.c_double)
    q = lc_quad(phi.size, mu.size, phi.ctypes.data_as(dp), mu.ctypes.data_as(dp), omega.ctypes.data_as(dp))
    h = C.c_void_p()
    _check(_lib.lc_build_rays(C.byref(g), C.byref(q), float(h_moc), int(mode), _stream(stream), C.byref(h)))
    return Rays(h, int(nx), int(ny), phi.size, mu.size)


def lc_rays_export(rays: Rays):
    """Host copies: (ray_off, seg_off, cell, len, width, face)."""
    ro = np.zeros(rays.n_pairs + 1, np.int32)
    so = np.zeros(rays.n_rays + 1, np.int32)
    ce = np.zeros(rays.n_segments, np.int32)
    ln = np.zeros(rays.n_segments, np.float64)
    wd = np.zeros(rays.n_rays, np.float64)
    fc = np.zeros((rays.n_rays, 2), np.int32)
    _check(_lib.lc_rays_export(rays.handle, ro.ctypes.data, so.ctypes.data, ce.ctypes.data,
                               ln.ctypes.data, wd.ctypes.data, fc.ctypes.data))
    return ro, so, ce, ln, wd, fc


class Plan:
    """Owning wrapper of an ``lc_plan_t`` handle (keeps its rays alive)."""

    def __init__(self, rays: Rays, G: int, prec: int):
        h = C.c_void_p()
        _check(_lib.lc_plan_create(rays.handle, int(G), int(prec), C.byref(h)))
        self.handle = h
        self.rays = rays
        self.G = int(G)
        self.prec = int(prec)
        self.state_bytes = int(_lib.lc_state_bytes(h))
        r = rays
        self.n_state = r.n_segments * 2 * r.n_pol * self.G
        self.n_field = r.cells * self.G
        self.n_in = r.nb * r.M * self.G
        self.n_exit = r.n_rays * 2 * r.n_pol * self.G

    def free(self):
        if self.handle:
            _check(_lib.lc_plan_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def new_state(self):
        import torch
        return torch.empty(self.state_bytes, dtype=torch.uint8, device="cuda")


def lc_plan_create(rays: Rays, G: int, prec: int) -> Plan:
    return Plan(rays, G, prec)


def lc_state_fill(plan: Plan, field, state, stream=None):
    _check(_lib.lc_state_fill(plan.handle, _dev(field, plan.n_field, name="field"),
                              _bytes(state, plan.state_bytes, "state"), _stream(stream)))


def lc_state_export(plan: Plan, state, out, stream=None):
    _check(_lib.lc_state_export(plan.handle, _bytes(state, plan.state_bytes, "state"),
                                _dev(out, plan.n_state, name="out"), _stream(stream)))


def lc_state_import(plan: Plan, src, state, stream=None):
    _check(_lib.lc_state_import(plan.handle, _dev(src, plan.n_state, name="src"),
                                _bytes(state, plan.state_bytes, "state"), _stream(stream)))


def lc_sweep(plan: Plan, kappa, planck, c_dt, state_prev, state_new, I_in, I_exit=None, stream=None):
    _check(_lib.lc_sweep(plan.handle, _dev(kappa, plan.n_field, name="kappa"),
                         _dev(planck, plan.n_field, name="planck"), float(c_dt),
                         _bytes(state_prev, plan.state_bytes, "state_prev"),
                         _bytes(state_new, plan.state_bytes, "state_new"),
                         _dev(I_in, plan.n_in, name="I_in"),
                         _dev(I_exit, plan.n_exit, name="I_exit", optional=True), _stream(stream)))


def lc_sweep_noalloc(plan: Plan, kappa, planck, c_dt, state_prev, state_new, I_in, I_exit=None, stream=None):
    _check(_lib.lc_sweep_noalloc(plan.handle, _dev(kappa, plan.n_field, name="kappa"),
                                 _dev(planck, plan.n_field, name="planck"), float(c_dt),
                                 _bytes(state_prev, plan.state_bytes, "state_prev"),
                                 _bytes(state_new, plan.state_bytes, "state_new"),
                                 _dev(I_in, plan.n_in, name="I_in"),
                                 _dev(I_exit, plan.n_exit, name="I_exit", optional=True), _stream(stream)))


def lc_moments(plan: Plan, state, c, E=None, F=None, f=None, bnd=None, I_exit=None, I_in=None,
               stream=None):
    r = plan.rays
    _check(_lib.lc_moments(plan.handle, _bytes(state, plan.state_bytes, "state"),
                           _dev(I_exit, plan.n_exit, name="I_exit", optional=True),
                           _dev(I_in, plan.n_in, name="I_in", optional=True), float(c),
                           _dev(E, plan.n_field, name="E", optional=True),
                           _dev(F, 2 * plan.n_field, name="F", optional=True),
                           _dev(f, 4 * plan.n_field, name="f", optional=True),
                           _dev(bnd, plan.G * r.nb * 8, name="bnd", optional=True), _stream(stream)))


def n_interior_faces(rays) -> int:
    return (rays.nx - 1) * rays.ny + rays.nx * (rays.ny - 1)


def lc_plan_enable_faces(plan: Plan, stream=None):
    _check(_lib.lc_plan_enable_faces(plan.handle, _stream(stream)))


def lc_sweep_points(plan: Plan, kappa, planck, c_dt, state_prev, state_new, I_in, points, I_exit=None, stream=None):
    _check(_lib.lc_sweep_points(plan.handle, _dev(kappa, plan.n_field, name="kappa"),
                                _dev(planck, plan.n_field, name="planck"), float(c_dt),
                                _bytes(state_prev, plan.state_bytes, "state_prev"),
                                _bytes(state_new, plan.state_bytes, "state_new"), _dev(I_in, plan.n_in, name="I_in"),
                                _dev(I_exit, plan.n_exit, name="I_exit", optional=True),
                                _bytes(points, plan.state_bytes, "points"), _stream(stream)))


def lc_face_moments(plan: Plan, points, state, c, E=None, F=None, f=None, stream=None):
    n = n_interior_faces(plan.rays) * plan.G
    _check(_lib.lc_face_moments(plan.handle, _bytes(points, plan.state_bytes, "points"),
                                _bytes(state, plan.state_bytes, "state"), float(c),
                                _dev(E, n, name="E", optional=True), _dev(F, 2 * n, name="F", optional=True),
                                _dev(f, 4 * n, name="f", optional=True), _stream(stream)))


N_GREY = 13     # fields of lc_grey_closures, [N_GREY][cells]


def lc_grey_closures(plan: Plan, E, F, f, kappa, planck, out, stream=None):
    """Grey closures of every cell from the plan's cell moments (cell-major
    E, F, f as written by lc_moments) and [G][cells] kappa, planck."""
    n = plan.n_field
    _check(_lib.lc_grey_closures(plan.handle, _dev(E, n, name="E"), _dev(F, 2 * n, name="F"),
                                 _dev(f, 4 * n, name="f"), _dev(kappa, n, name="kappa"),
                                 _dev(planck, n, name="planck"), _dev(out, N_GREY * plan.rays.cells, name="out"),
                                 _stream(stream)))


def lc_grey_closures_dims(cells: int, G: int, E, F, f, kappa, planck, out, stream=None):
    """lc_grey_closures for moments of `cells` cells and G groups gathered
    from several plans (cell-major E, F, f; [G][cells] kappa, planck)."""
    n = int(cells) * int(G)
    _check(_lib.lc_grey_closures_dims(int(cells), int(G), _dev(E, n, name="E"), _dev(F, 2 * n, name="F"),
                                      _dev(f, 4 * n, name="f"), _dev(kappa, n, name="kappa"),
                                      _dev(planck, n, name="planck"), _dev(out, N_GREY * int(cells), name="out"),
                                      _stream(stream)))


def lc_plan_set_tuning(plan: Plan, sweep_unroll: int, moments_entries: int):
    t = lc_tuning_t(int(sweep_unroll), int(moments_entries))
    _check(_lib.lc_plan_set_tuning(plan.handle, C.byref(t)))


def lc_plan_set_sweep_residency(plan: Plan, capped: bool):
    _check(_lib.lc_plan_set_sweep_residency(plan.handle, int(bool(capped))))


def lc_plan_set_split(plan: Plan, chunk_steps: int):
    _check(_lib.lc_plan_set_split(plan.handle, int(chunk_steps)))


def lc_plan_set_moment_split(plan: Plan, mode: int):
    _check(_lib.lc_plan_set_moment_split(plan.handle, int(mode)))


def lc_plan_get_moment_split(plan: Plan) -> int:
    m = C.c_int32(0)
    _check(_lib.lc_plan_get_moment_split(plan.handle, C.byref(m)))
    return int(m.value)


def lc_plan_get_tuning(plan: Plan):
    t = lc_tuning_t()
    _check(_lib.lc_plan_get_tuning(plan.handle, C.byref(t)))
    return dict(sweep_unroll=t.sweep_unroll, moments_entries=t.moments_entries)


def lc_plan_profile(plan: Plan, enable: bool):
    _check(_lib.lc_plan_profile(plan.handle, int(bool(enable))))


def lc_plan_profile_read(plan: Plan):
    """(sweep_ms_total, sweep_launches, moments_ms_total, moments_launches)."""
    out = (C.c_double * 4)()
    _check(_lib.lc_plan_profile_read(plan.handle, out))
    return tuple(out)


def lc_step(plan: Plan, n_steps, kappa, planck, c_dt, c, state_a, state_b, I_in, I_exit=None,
            E=None, F=None, f=None, bnd=None, material_stride=0, stream=None):
    r = plan.rays
    n_mat = plan.n_field + (int(n_steps) - 1) * int(material_stride)
    _check(_lib.lc_step(plan.handle, int(n_steps), _dev(kappa, n_mat, name="kappa"),
                        _dev(planck, n_mat, name="planck"), int(material_stride), float(c_dt), float(c),
                        _bytes(state_a, plan.state_bytes, "state_a"),
                        _bytes(state_b, plan.state_bytes, "state_b"),
                        _dev(I_in, plan.n_in, name="I_in"),
                        _dev(I_exit, plan.n_exit, name="I_exit", optional=True),
                        _dev(E, plan.n_field, name="E", optional=True),
                        _dev(F, 2 * plan.n_field, name="F", optional=True),
                        _dev(f, 4 * plan.n_field, name="f", optional=True),
                        _dev(bnd, plan.G * r.nb * 8, name="bnd", optional=True), _stream(stream)))


class Batch:
    """Owning wrapper of an ``lc_batch_t`` handle; keeps the problems' plans
    and buffers alive."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep

    def free(self):
        if self.handle:
            _check(_lib.lc_batch_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def lc_batch_create(problems) -> Batch:
    """problems: list of dicts with keys plan, kappa, planck, material_stride,
    c_dt, state_a, state_b, I_in, I_exit and optionally E, F, f, bnd (device
    tensors sized as for lc_step)."""
    arr = (lc_problem_t * len(problems))()
    keep = []
    for i, p in enumerate(problems):
        plan = p["plan"]
        r = plan.rays
        n_steps = int(p.get("n_steps_max", 1))
        stride = int(p.get("material_stride", 0))
        n_mat = plan.n_field + (n_steps - 1) * stride
        arr[i] = lc_problem_t(
            plan.handle, _dev(p["kappa"], n_mat, name="kappa"), _dev(p["planck"], n_mat, name="planck"),
            stride, float(p["c_dt"]), _bytes(p["state_a"], plan.state_bytes, "state_a"),
            _bytes(p["state_b"], plan.state_bytes, "state_b"), _dev(p["I_in"], plan.n_in, name="I_in"),
            _dev(p["I_exit"], plan.n_exit, name="I_exit"),
            _dev(p.get("E"), plan.n_field, name="E", optional=True),
            _dev(p.get("F"), 2 * plan.n_field, name="F", optional=True),
            _dev(p.get("f"), 4 * plan.n_field, name="f", optional=True),
            _dev(p.get("bnd"), plan.G * r.nb * 8, name="bnd", optional=True))
        keep.append(p)
    h = C.c_void_p()
    _check(_lib.lc_batch_create(len(problems), arr, C.byref(h)))
    return Batch(h, keep)


def lc_batch_step(batch: Batch, n_steps: int, c: float, stream=None):
    _check(_lib.lc_batch_step(batch.handle, int(n_steps), float(c), _stream(stream)))


def lc_batch_profile(batch: Batch, enable: bool):
    _check(_lib.lc_batch_profile(batch.handle, int(bool(enable))))


def lc_batch_profile_read(batch: Batch):
    """(prologue_ms, n, sweep_ms, n, moments_ms, n) totals since the last read."""
    out = (C.c_double * 6)()
    _check(_lib.lc_batch_profile_read(batch.handle, out))
    return tuple(out)



class Loqd:
    """Owning wrapper of an ``lc_loqd_t`` handle (multigroup LOQD solver of
    an nx x ny grid for G groups)."""

    def __init__(self, nx, ny, lx, ly, G):
        h = C.c_void_p()
        _check(_lib.lc_loqd_create(int(nx), int(ny), float(lx), float(ly), int(G), C.byref(h)))
        self.handle = h
        self.nx, self.ny, self.G = int(nx), int(ny), int(G)
        self.cells = self.nx * self.ny
        self.n_interior = (self.nx - 1) * self.ny + self.nx * (self.ny - 1)
        self.nb = 2 * (self.nx + self.ny)
        self.nf = self.n_interior + self.nb

    def free(self):
        if self.handle:
            _check(_lib.lc_loqd_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def lc_loqd_solve(h: Loqd, c, c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bnd, E_cell, E_face, F_face,
                  rtol=1e-13, max_iter=20000, stream=None):
    """Returns (iterations, per-group relative residuals)."""
    G, N, nf = h.G, h.cells, h.nf
    it = C.c_int32(0)
    res = np.zeros(G)
    _check(_lib.lc_loqd_solve(h.handle, float(c), float(c_dt), _dev(kappa, G * N, name="kappa"),
                              _dev(planck, G * N, name="planck"), _dev(E_prev, G * N, name="E_prev"),
                              _dev(F_prev, G * nf, name="F_prev"), _dev(f_cell, 4 * G * N, name="f_cell"),
                              _dev(f_face, 4 * G * h.n_interior, name="f_face", optional=h.n_interior == 0),
                              _dev(bnd, 8 * G * h.nb, name="bnd"), _dev(E_cell, G * N, name="E_cell"),
                              _dev(E_face, G * nf, name="E_face"), _dev(F_face, G * nf, name="F_face"),
                              float(rtol), int(max_iter), C.byref(it), res.ctypes.data, _stream(stream)))
    return int(it.value), res


def lc_loqd_solve_general(h: Loqd, c, c_dt, sigma, source, k_side, eta_side, F_prev, f_cell, f_face, bc, E_cell,
                          E_face, F_face, rtol=1e-13, max_iter=20000, stream=None):
    """General form (the handle's G groups).  Returns (iterations, residuals)."""
    G, N, nf = h.G, h.cells, h.nf
    it = C.c_int32(0)
    res = np.zeros(G)
    _check(_lib.lc_loqd_solve_general(h.handle, float(c), float(c_dt), _dev(sigma, G * N, name="sigma"),
                                      _dev(source, G * N, name="source"), _dev(k_side, 4 * G * N, name="k_side"),
                                      _dev(eta_side, 4 * G * N, name="eta_side"), _dev(F_prev, G * nf, name="F_prev"),
                                      _dev(f_cell, 3 * G * N, name="f_cell"), _dev(f_face, 3 * G * nf, name="f_face"),
                                      _dev(bc, 3 * G * h.nb, name="bc"), _dev(E_cell, G * N, name="E_cell"),
                                      _dev(E_face, G * nf, name="E_face"), _dev(F_face, G * nf, name="F_face"),
                                      float(rtol), int(max_iter), C.byref(it), res.ctypes.data, _stream(stream)))
    return int(it.value), res


def lc_loqd_grey_coefficients(h: Loqd, c, c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bnd, E_cell, E_face,
                              F_face, out, stream=None):
    """out: dict of device tensors sigma, source, E_prev [cells]; k_side,
    eta_side [4 cells]; F_prev [nf]; f_cell [3 cells]; f_face [3 nf];
    bc [3 nb]; optionally kappa_E, kappa_B [cells] (the grey coefficients
    are written there)."""
    G, N, nf = h.G, h.cells, h.nf
    _check(_lib.lc_loqd_grey_coefficients(
        h.handle, float(c), float(c_dt), _dev(kappa, G * N, name="kappa"), _dev(planck, G * N, name="planck"),
        _dev(E_prev, G * N, name="E_prev"), _dev(F_prev, G * nf, name="F_prev"),
        _dev(f_cell, 4 * G * N, name="f_cell"),
        _dev(f_face, 4 * G * h.n_interior, name="f_face", optional=h.n_interior == 0),
        _dev(bnd, 8 * G * h.nb, name="bnd"), _dev(E_cell, G * N, name="E_cell"), _dev(E_face, G * nf, name="E_face"),
        _dev(F_face, G * nf, name="F_face"), _dev(out["sigma"], N, name="sigma"), _dev(out["source"], N, name="source"),
        _dev(out["k_side"], 4 * N, name="k_side"), _dev(out["eta_side"], 4 * N, name="eta_side"),
        _dev(out["F_prev"], nf, name="F_prev out"), _dev(out["f_cell"], 3 * N, name="f_cell out"),
        _dev(out["f_face"], 3 * nf, name="f_face out"), _dev(out["bc"], 3 * h.nb, name="bc out"),
        _dev(out["E_prev"], N, name="E_prev out"), _dev(out.get("kappa_E"), N, name="kappa_E", optional=True),
        _dev(out.get("kappa_B"), N, name="kappa_B", optional=True), _stream(stream)))


def lc_loqd_grey_meb(h: Loqd, c, c_dt, kappa_E, kappa_B, E_prev, k_side, eta_side, F_prev, f_cell, f_face, bc,
                     T_prev, c_v, a_R, T, E_cell, E_face, F_face, newton_tol=1e-10, max_newton=50, rtol=1e-13,
                     max_iter=20000, stream=None):
    """The grey problem with the energy balance (the handle's G independent
    problems).  T is the first iterate on entry and the result on return.
    Returns (Newton iterations, BiCGSTAB iterations, last residuals)."""
    G, N, nf = h.G, h.cells, h.nf
    nit, it = C.c_int32(0), C.c_int32(0)
    res = np.zeros(G)
    _check(_lib.lc_loqd_grey_meb(
        h.handle, float(c), float(c_dt), _dev(kappa_E, G * N, name="kappa_E"), _dev(kappa_B, G * N, name="kappa_B"),
        _dev(E_prev, G * N, name="E_prev"), _dev(k_side, 4 * G * N, name="k_side"),
        _dev(eta_side, 4 * G * N, name="eta_side"), _dev(F_prev, G * nf, name="F_prev"),
        _dev(f_cell, 3 * G * N, name="f_cell"), _dev(f_face, 3 * G * nf, name="f_face"),
        _dev(bc, 3 * G * h.nb, name="bc"), _dev(T_prev, G * N, name="T_prev"), float(c_v), float(a_R),
        _dev(T, G * N, name="T"), _dev(E_cell, G * N, name="E_cell"), _dev(E_face, G * nf, name="E_face"),
        _dev(F_face, G * nf, name="F_face"), float(newton_tol), int(max_newton), float(rtol), int(max_iter),
        C.byref(nit), C.byref(it), res.ctypes.data, _stream(stream)))
    return int(nit.value), int(it.value), res



def lc_set_alloc_limit(nbytes):
    """Device allocations of the library above nbytes fail with LC_ERR_ALLOC (0: no limit)."""
    _check(_lib.lc_set_alloc_limit(int(nbytes)))


def lc_set_validation(enable):
    """Check material and boundary inputs for non-finite or negative values before sweeps."""
    _check(_lib.lc_set_validation(int(bool(enable))))


def lc_loqd_set_solver(h: Loqd, mode):
    """0 by size, 1 one workgroup per group, 2 many blocks per group."""
    _check(_lib.lc_loqd_set_solver(h.handle, int(mode)))


def lc_loqd_set_warm_start(h: Loqd, enable=True):
    _check(_lib.lc_loqd_set_warm_start(h.handle, int(bool(enable))))


class Mlqd:
    """Owning wrapper of an ``lc_mlqd_t`` handle: multilevel time steps on
    the Fleck-Cummings material for a plan (kept alive here)."""

    def __init__(self, plan: Plan, nu, edges, c, c_v, a_R):
        nu = np.ascontiguousarray(nu, dtype=np.float64)
        edges = np.ascontiguousarray(edges, dtype=np.float64)
        if nu.size != plan.G or edges.size != plan.G + 1:
            raise ValueError("nu needs G values and edges G + 1")
        h = C.c_void_p()
        _check(_lib.lc_mlqd_create(plan.handle, nu.ctypes.data, edges.ctypes.data, float(c), float(c_v), float(a_R),
                                   C.byref(h)))
        self.handle = h
        self.plan = plan
        self.G = plan.G
        r = plan.rays
        self.cells = r.cells
        self.n_interior = (r.nx - 1) * r.ny + r.nx * (r.ny - 1)
        self.nb = 2 * (r.nx + r.ny)
        self.nf = self.n_interior + self.nb

    def free(self):
        if self.handle:
            _check(_lib.lc_mlqd_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def lc_mlqd_set_acceleration(h: Mlqd, depth):
    _check(_lib.lc_mlqd_set_acceleration(h.handle, int(depth)))


def lc_mlqd_material(h: Mlqd, T, kappa, planck, stream=None):
    G, N = h.G, h.cells
    _check(_lib.lc_mlqd_material(h.handle, _dev(T, N, name="T"), _dev(kappa, G * N, name="kappa"),
                                 _dev(planck, G * N, name="planck"), _stream(stream)))


def lc_mlqd_step(h: Mlqd, c_dt, state_prev, state_new, I_in, T_prev, E_prev, F_prev, T, E_cell, E_face, F_face,
                 E_grey=None, eps=1e-12, max_outer=60, max_inner=1000, stream=None):
    """Returns (outer iterations, inner iterations, (dT, dE))."""
    G, N, nf = h.G, h.cells, h.nf
    nbytes = h.plan.state_bytes
    so, si = C.c_int32(0), C.c_int32(0)
    ch = np.zeros(2)
    _check(_lib.lc_mlqd_step(
        h.handle, float(c_dt), _bytes(state_prev, nbytes, "state_prev"), _bytes(state_new, nbytes, "state_new"),
        _dev(I_in, h.plan.n_in, name="I_in"), _dev(T_prev, N, name="T_prev"), _dev(E_prev, G * N, name="E_prev"),
        _dev(F_prev, G * nf, name="F_prev"), _dev(T, N, name="T"), _dev(E_cell, G * N, name="E_cell"),
        _dev(E_face, G * nf, name="E_face"), _dev(F_face, G * nf, name="F_face"),
        _dev(E_grey, N, name="E_grey", optional=True), float(eps), int(max_outer), int(max_inner), C.byref(so),
        C.byref(si), ch.ctypes.data, _stream(stream)))
    return int(so.value), int(si.value), (float(ch[0]), float(ch[1]))