"""Python binding of the gfx950 library liblbmep.so (C ABI in include/lbmep.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  The raw functions keep the C names (``lbmep_create``,
``lbmep_step``, ...); ``Lattice`` is a thin object wrapper over them.
Host arrays are numpy arrays; device arrays are torch CUDA tensors (their
``data_ptr`` is passed with ``on_device = 1``).  PyTorch is used only for
device memory and streams.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblbmep.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENONFINITE, EBUSY = 0, -1, -2, -3, -4, -5, -6
FP64, FP32DEV, FP16DEV = 0, 1, 2
FLUID, WALL, OBST, NEAR = 0, 1, 2, 3
DTYPE_F64, DTYPE_F32 = 0, 1

PRECISIONS = {"fp64": FP64, "fp32dev": FP32DEV, "fp16dev": FP16DEV}


class LbmepError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbmep error {code}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("periodic", ctypes.c_int32 * 3),
        ("nu", ctypes.c_double), ("magic", ctypes.c_double),
        ("precision", ctypes.c_int32), ("move_particles", ctypes.c_int32),
        ("device", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
    ]


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int32), ("max_slots", ctypes.c_int32),
        ("chunk_steps", ctypes.c_int32), ("max_queue", ctypes.c_int32),
        ("hbm_budget", ctypes.c_size_t),
    ]


class Request(ctypes.Structure):
    _fields_ = [
        ("cfg", Config),
        ("flags", ctypes.c_void_p),
        ("n", ctypes.c_int32), ("steps", ctypes.c_int32),
        ("X", ctypes.c_void_p), ("R", ctypes.c_void_p), ("U", ctypes.c_void_p),
        ("W", ctypes.c_void_p),
        ("rho_e", ctypes.c_void_p),
        ("rho_e_dtype", ctypes.c_int32), ("keep_fields", ctypes.c_int32),
        ("E", ctypes.c_double * 3),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
        ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
        ("queued", ctypes.c_int32), ("resident", ctypes.c_int32),
        ("chunks", ctypes.c_uint64), ("steps", ctypes.c_uint64),
        ("packed_launches", ctypes.c_uint64),
        ("cell_updates", ctypes.c_double), ("cell_updates_done", ctypes.c_double),
        ("bytes_reserved", ctypes.c_size_t), ("bytes_in_use", ctypes.c_size_t),
        ("budget", ctypes.c_size_t),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

# exported symbols and their ctypes signatures
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_SIGS = {
    "lbmep_last_error": (ctypes.c_char_p, []),
    "lbmep_create": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_void_p)]),
    "lbmep_destroy": (ctypes.c_int, [_P]),
    "lbmep_set_flags": (ctypes.c_int, [_P, _P, ctypes.c_int]),
    "lbmep_set_particles": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P]),
    "lbmep_set_force": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int]),
    "lbmep_set_charge_force": (ctypes.c_int, [_P, _P, ctypes.c_int, _D, ctypes.c_int]),
    "lbmep_set_potential_force": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_double, _D, _D,
                                                 ctypes.c_int]),
    "lbmep_set_potential_solver": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double,
                                                  ctypes.c_int32, ctypes.c_double,
                                                  ctypes.c_int32]),
    "lbmep_solve_potential": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), _D]),
    "lbmep_get_solver_stats": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), _D]),
    "lbmep_get_solver_shape": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "lbmep_get_invariants_noalloc": (ctypes.c_int, [_P, ctypes.c_void_p]),
    "lbmep_get_potential": (ctypes.c_int, [_P, _P, ctypes.c_int]),
    "lbmep_set_dynamics": (ctypes.c_int, [_P, ctypes.c_double, _P, _D]),
    "lbmep_set_free_slip": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "lbmep_get_particles": (ctypes.c_int, [_P, _D, _D, _D]),
    "lbmep_init_equilibrium": (ctypes.c_int, [_P, ctypes.c_double, _D]),
    "lbmep_set_pdfs": (ctypes.c_int, [_P, _P, ctypes.c_int]),
    "lbmep_get_pdfs": (ctypes.c_int, [_P, _P, ctypes.c_int]),
    "lbmep_step": (ctypes.c_int, [_P, ctypes.c_int32]),
    "lbmep_sync": (ctypes.c_int, [_P]),
    "lbmep_get_macro": (ctypes.c_int, [_P, _P, _P, ctypes.c_int]),
    "lbmep_get_particle_ft": (ctypes.c_int, [_P, _P, _P]),
    "lbmep_get_map": (ctypes.c_int, [_P, _P, _P]),
    "lbmep_get_invariants": (ctypes.c_int, [_P, _D]),
    "lbmep_get_time": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "lbmep_set_timing": (ctypes.c_int, [_P, ctypes.c_int]),
    "lbmep_get_timing": (ctypes.c_int, [_P, _D, ctypes.POINTER(ctypes.c_int64)]),
    "lbmep_save_state": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "lbmep_load_state": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "lbmep_get_particle_count": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "lbmep_footprint": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.c_int32, ctypes.c_double,
                                       ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "lbmep_copy_reference": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                            ctypes.c_void_p]),
    "lbmep_server_create": (ctypes.c_int, [ctypes.POINTER(ServerConfig),
                                           ctypes.POINTER(ctypes.c_void_p)]),
    "lbmep_server_destroy": (ctypes.c_int, [_P]),
    "lbmep_server_request_footprint": (ctypes.c_int, [ctypes.POINTER(Request),
                                                      ctypes.POINTER(ctypes.c_size_t)]),
    "lbmep_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(Request),
                                           ctypes.POINTER(ctypes.c_uint64)]),
    "lbmep_server_poll": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32)]),
    "lbmep_server_result": (ctypes.c_int, [_P, ctypes.c_uint64, _P, _P, _D, _D]),
    "lbmep_server_fields": (ctypes.c_int, [_P, ctypes.c_uint64, _P, _P]),
    "lbmep_server_release": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "lbmep_server_get_stats": (ctypes.c_int, [_P, ctypes.POINTER(ServerStats)]),
    "lbmep_server_now": (ctypes.c_int, [_P, _D]),
}


def lib():
    """Load liblbmep.so; raise if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with paper_1708_08741_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(rc):
    if rc != OK:
        msg = lib().lbmep_last_error().decode(errors="replace")
        raise LbmepError(rc, msg)
    return rc


def _ptr(a):
    """(pointer, on_device) of a numpy array or a torch tensor."""
    if isinstance(a, np.ndarray):
        assert a.flags.c_contiguous
        return ctypes.c_void_p(a.ctypes.data), 0
    # torch tensor
    assert a.is_contiguous()
    return ctypes.c_void_p(a.data_ptr()), 1 if a.is_cuda else 0


def _dp(a):
    return a.ctypes.data_as(_D)


def make_config(shape, periodic=(True, True, True), nu=1.0 / 6.0, magic=3.0 / 16.0,
                precision=FP64, move_particles=False, device=0, stream=None):
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    c = Config()
    c.nx, c.ny, c.nz = (int(s) for s in shape)
    for k in range(3):
        c.periodic[k] = 1 if periodic[k] else 0
    c.nu = float(nu)
    c.magic = float(magic)
    c.precision = int(precision)
    c.move_particles = 1 if move_particles else 0
    c.device = int(device)
    c.reserved = 0
    c.stream = stream
    return c


def copy_reference(dst, src, stream=None):
    """The achievable-bandwidth reference copy (lbmep_copy_reference) of two
    equally sized device tensors; asynchronous on `stream` (a hipStream_t
    handle, None = the default stream)."""
    n = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() >= n
    _check(lib().lbmep_copy_reference(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                      n, ctypes.c_void_p(stream or 0)))


def footprint(shape, precision=FP64, n_particles=0, with_charge=False, r_max=8.0, **kw):
    cfg = make_config(shape, precision=precision, **kw)
    out = ctypes.c_size_t(0)
    _check(lib().lbmep_footprint(ctypes.byref(cfg), int(n_particles), float(r_max),
                                 1 if with_charge else 0, ctypes.byref(out)))
    return out.value


class Lattice:
    """One lattice of the GPU library.  Host arrays use numpy (z, y, x) order."""

    def __init__(self, shape, periodic=(True, True, True), nu=1.0 / 6.0, magic=3.0 / 16.0,
                 precision=FP64, move_particles=False, device=0, stream=None):
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        self.cfg = make_config(shape, periodic, nu, magic, precision, move_particles, device,
                               stream)
        self.shape = tuple(int(s) for s in shape)
        nx, ny, nz = self.shape
        self.N = nx * ny * nz
        self.np = 0
        h = ctypes.c_void_p()
        _check(lib().lbmep_create(ctypes.byref(self.cfg), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().lbmep_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_flags(self, flags):
        if isinstance(flags, np.ndarray):
            flags = np.ascontiguousarray(flags, dtype=np.uint8).reshape(-1)
        p, dev = _ptr(flags)
        _check(lib().lbmep_set_flags(self._h, p, dev))

    def set_particles(self, X, R, U, W=None):
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1)
        R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1)
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(-1)
        n = len(R)
        Wp = None
        if W is not None:
            W = np.ascontiguousarray(W, dtype=np.float64).reshape(-1)
            Wp = W.ctypes.data
        _check(lib().lbmep_set_particles(self._h, n, X.ctypes.data, R.ctypes.data, U.ctypes.data,
                                         Wp))
        self.np = n

    def set_force(self, fb):
        if isinstance(fb, np.ndarray):
            fb = np.ascontiguousarray(fb)
            dt = DTYPE_F32 if fb.dtype == np.float32 else DTYPE_F64
            fb = fb.astype(np.float32 if dt == DTYPE_F32 else np.float64, copy=False).reshape(-1)
        else:
            import torch
            dt = DTYPE_F32 if fb.dtype == torch.float32 else DTYPE_F64
        p, dev = _ptr(fb)
        _check(lib().lbmep_set_force(self._h, p, dt, dev))

    def set_charge_force(self, rho_e, E):
        if isinstance(rho_e, np.ndarray):
            rho_e = np.ascontiguousarray(rho_e)
            dt = DTYPE_F32 if rho_e.dtype == np.float32 else DTYPE_F64
            rho_e = rho_e.astype(np.float32 if dt == DTYPE_F32 else np.float64,
                                 copy=False).reshape(-1)
        else:
            import torch
            dt = DTYPE_F32 if rho_e.dtype == torch.float32 else DTYPE_F64
        Ea = np.array(E, dtype=np.float64)
        p, dev = _ptr(rho_e)
        _check(lib().lbmep_set_charge_force(self._h, p, dt, _dp(Ea), dev))

    def set_potential_force(self, psi, kappa2_eps, E, zeta=None):
        """Body force rho_e(psi) (E - grad psi) computed in the sweep from the
        EDL potential psi (nz, ny, nx) with rho_e = -kappa2_eps psi; zeta =
        per-particle surface potential (None: psi's value at obstacle cells)."""
        if isinstance(psi, np.ndarray):
            psi = np.ascontiguousarray(psi)
            dt = DTYPE_F32 if psi.dtype == np.float32 else DTYPE_F64
            psi = psi.astype(np.float32 if dt == DTYPE_F32 else np.float64,
                             copy=False).reshape(-1)
        else:
            import torch
            dt = DTYPE_F32 if psi.dtype == torch.float32 else DTYPE_F64
        Ea = np.array(E, dtype=np.float64)
        zp = None
        if zeta is not None:
            za = np.ascontiguousarray(zeta, dtype=np.float64).reshape(-1)
            zp = _dp(za)
        p, dev = _ptr(psi)
        _check(lib().lbmep_set_potential_force(self._h, p, dt, float(kappa2_eps), _dp(Ea), zp,
                                               dev))

    def set_potential_solver(self, kappa2, omega=1.7, max_iter=0, rf=0.0, check_every=1):
        """Red-black SOR for the Debye-Hueckel equation of the potential;
        max_iter > 0 also solves before every step."""
        _check(lib().lbmep_set_potential_solver(self._h, float(kappa2), float(omega),
                                                int(max_iter), float(rf), int(check_every)))

    def solve_potential(self):
        """One solve on the current map: (iterations, res0, res)."""
        it = ctypes.c_int32(0)
        res = np.zeros(2)
        _check(lib().lbmep_solve_potential(self._h, ctypes.byref(it), _dp(res)))
        return it.value, float(res[0]), float(res[1])

    def solver_stats(self):
        it = ctypes.c_int32(0)
        res = np.zeros(2)
        _check(lib().lbmep_get_solver_stats(self._h, ctypes.byref(it), _dp(res)))
        return it.value, float(res[0]), float(res[1])

    def solver_shape(self):
        """(one_pass, rows per thread, planes per workgroup, wavefronts)."""
        out = (ctypes.c_int32 * 4)()
        _check(lib().lbmep_get_solver_shape(self._h, out))
        return tuple(int(v) for v in out)

    def potential(self, out=None):
        nx, ny, nz = self.shape
        if out is None:
            out = np.zeros((nz, ny, nx))
        p, dev = _ptr(out)
        _check(lib().lbmep_get_potential(self._h, p, dev))
        return out

    def set_free_slip(self, faces):
        """Free-slip faces (x-, x+, y-, y+, z-, z+), non-periodic axes only."""
        f = (ctypes.c_int32 * 6)(*[1 if v else 0 for v in faces])
        _check(lib().lbmep_set_free_slip(self._h, f))

    def set_dynamics(self, rho_p, q=None, E=(0.0, 0.0, 0.0)):
        """Newton-Euler dynamics of the (moving) particles: density rho_p,
        charges q (None: uncharged), applied field E for the forces q E."""
        qp = None
        if q is not None:
            qa = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
            qp = ctypes.c_void_p(qa.ctypes.data)
        Ea = np.array(E, dtype=np.float64)
        _check(lib().lbmep_set_dynamics(self._h, float(rho_p), qp, _dp(Ea)))

    def particles(self):
        """Current positions, velocities, angular velocities, (n, 3) each."""
        X = np.zeros((self.np, 3))
        U = np.zeros((self.np, 3))
        Wv = np.zeros((self.np, 3))
        _check(lib().lbmep_get_particles(self._h, _dp(X), _dp(U), _dp(Wv)))
        return X, U, Wv

    def init_equilibrium(self, rho=1.0, u=(0.0, 0.0, 0.0)):
        ua = np.array(u, dtype=np.float64)
        _check(lib().lbmep_init_equilibrium(self._h, float(rho), _dp(ua)))

    def set_pdfs(self, f):
        if isinstance(f, np.ndarray):
            f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        p, dev = _ptr(f)
        _check(lib().lbmep_set_pdfs(self._h, p, dev))

    def get_pdfs(self, out=None):
        nx, ny, nz = self.shape
        if out is None:
            out = np.zeros((19, nz, ny, nx))
        p, dev = _ptr(out)
        _check(lib().lbmep_get_pdfs(self._h, p, dev))
        return out

    def step(self, n=1):
        _check(lib().lbmep_step(self._h, int(n)))

    def sync(self):
        _check(lib().lbmep_sync(self._h))

    @property
    def time(self):
        t = ctypes.c_int64(0)
        _check(lib().lbmep_get_time(self._h, ctypes.byref(t)))
        return t.value

    def macro(self):
        nx, ny, nz = self.shape
        rho = np.zeros((nz, ny, nx))
        u = np.zeros((3, nz, ny, nx))
        _check(lib().lbmep_get_macro(self._h, rho.ctypes.data, u.ctypes.data, 0))
        return rho, u

    def macro_device(self, rho, u):
        _check(lib().lbmep_get_macro(self._h, ctypes.c_void_p(rho.data_ptr()),
                                     ctypes.c_void_p(u.data_ptr()), 1))

    def ft(self):
        F = np.zeros((self.np, 3))
        M = np.zeros((self.np, 3))
        if self.np:
            _check(lib().lbmep_get_particle_ft(self._h, F.ctypes.data, M.ctypes.data))
        return F, M

    def map(self):
        nx, ny, nz = self.shape
        fl = np.zeros((nz, ny, nx), dtype=np.uint8)
        ow = np.zeros((nz, ny, nx), dtype=np.int32)
        _check(lib().lbmep_get_map(self._h, fl.ctypes.data, ow.ctypes.data))
        return fl, ow

    def invariants(self):
        out = np.zeros(4)
        _check(lib().lbmep_get_invariants(self._h, _dp(out)))
        return out

    def invariants_noalloc(self, out):
        """lbmep_get_invariants_noalloc: the FP64 sums into `out` (a device
        tensor of 4 float64), asynchronous on the lattice's stream."""
        assert out.is_cuda and out.dtype.itemsize == 8 and out.numel() >= 4
        _check(lib().lbmep_get_invariants_noalloc(self._h, ctypes.c_void_p(out.data_ptr())))

    def set_timing(self, enable=True):
        _check(lib().lbmep_set_timing(self._h, 1 if enable else 0))

    def get_timing(self):
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        _check(lib().lbmep_get_timing(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def save(self, path):
        _check(lib().lbmep_save_state(self._h, str(path).encode()))

    def load(self, path):
        _check(lib().lbmep_load_state(self._h, str(path).encode()))
        n = ctypes.c_int32(0)
        _check(lib().lbmep_get_particle_count(self._h, ctypes.byref(n)))
        self.np = n.value


def from_workload(wl, precision=None, device=0, stream=None, force_dtype=None):
    """Set up a GPU lattice for a workloads.Workload."""
    prec = PRECISIONS[precision or wl.precision]
    L = Lattice(wl.shape, wl.periodic, wl.nu, wl.magic, prec, wl.moving, device, stream)
    L.set_flags(wl.flags)
    if force_dtype is None:
        force_dtype = np.float64 if prec == FP64 else np.float32
    if wl.rho_e is not None:
        L.set_charge_force(wl.rho_e.astype(force_dtype), wl.E)
    elif wl.fb is not None:
        L.set_force(wl.fb.astype(force_dtype))
    L.init_equilibrium(1.0, (0.0, 0.0, 0.0))
    L.set_particles(wl.X, wl.R, wl.U, wl.W)
    return L


class Server:
    """Request server of the library (lbmep_server_*): continuous batching of
    independent simulations with packed launches.  Request inputs are numpy
    arrays; they are copied by submit."""

    def __init__(self, hbm_budget, max_slots=32, chunk_steps=20, max_queue=100000, device=0):
        c = ServerConfig()
        c.device = int(device)
        c.max_slots = int(max_slots)
        c.chunk_steps = int(chunk_steps)
        c.max_queue = int(max_queue)
        c.hbm_budget = int(hbm_budget)
        h = ctypes.c_void_p()
        _check(lib().lbmep_server_create(ctypes.byref(c), ctypes.byref(h)))
        self._h = h
        self.meta = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().lbmep_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _request(shape, X=None, R=None, U=None, W=None, steps=1, rho_e=None, E=(0, 0, 0),
                 flags=None, periodic=(True, True, True), nu=1.0 / 6.0, magic=3.0 / 16.0,
                 precision=FP32DEV, moving=True, keep_fields=False):
        q = Request()
        q.cfg = make_config(shape, periodic, nu, magic, precision, moving, 0, None)
        keep = []
        X = np.zeros((0, 3)) if X is None else X
        R = np.zeros(0) if R is None else R
        U = np.zeros((0, 3)) if U is None else U
        arrs = {}
        for k, a in (("X", X), ("R", R), ("U", U), ("W", W)):
            if a is None:
                continue
            a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
            keep.append(a)
            arrs[k] = a.ctypes.data
        q.n = len(np.asarray(R).reshape(-1))
        q.steps = int(steps)
        q.X, q.R, q.U = arrs["X"], arrs["R"], arrs["U"]
        q.W = arrs.get("W")
        if flags is not None:
            fl = np.ascontiguousarray(flags, dtype=np.uint8).reshape(-1)
            keep.append(fl)
            q.flags = fl.ctypes.data
        if rho_e is not None:
            re = np.ascontiguousarray(rho_e)
            if re.dtype not in (np.float32, np.float64):
                re = re.astype(np.float64)
            re = re.reshape(-1)
            keep.append(re)
            q.rho_e = re.ctypes.data
            q.rho_e_dtype = DTYPE_F32 if re.dtype == np.float32 else DTYPE_F64
            for k in range(3):
                q.E[k] = float(E[k])
        q.keep_fields = 1 if keep_fields else 0
        return q, keep

    @staticmethod
    def request_footprint(shape, **kw):
        q, keep = Server._request(shape, **kw)
        out = ctypes.c_size_t(0)
        _check(lib().lbmep_server_request_footprint(ctypes.byref(q), ctypes.byref(out)))
        return out.value

    def submit(self, shape, **kw):
        """Queue one simulation; returns its id."""
        q, keep = self._request(shape, **kw)
        rid = ctypes.c_uint64(0)
        _check(lib().lbmep_server_submit(self._h, ctypes.byref(q), ctypes.byref(rid)))
        R = kw.get("R")
        self.meta[rid.value] = dict(shape=tuple(shape), n=q.n, steps=q.steps)
        return rid.value

    def poll(self, cap=1024):
        ids = (ctypes.c_uint64 * cap)()
        n = ctypes.c_int32(0)
        _check(lib().lbmep_server_poll(self._h, ids, cap, ctypes.byref(n)))
        return [ids[i] for i in range(n.value)]

    def result(self, rid):
        """(F, M, invariants, (t_submit, t_admit, t_done)) of a finished request."""
        n = self.meta[rid]["n"]
        F = np.zeros((n, 3))
        M = np.zeros((n, 3))
        inv = np.zeros(4)
        t = np.zeros(3)
        _check(lib().lbmep_server_result(self._h, rid, F.ctypes.data, M.ctypes.data, _dp(inv),
                                         _dp(t)))
        return F, M, inv, tuple(t)

    def fields(self, rid):
        nx, ny, nz = self.meta[rid]["shape"]
        rho = np.zeros((nz, ny, nx))
        u = np.zeros((3, nz, ny, nx))
        _check(lib().lbmep_server_fields(self._h, rid, rho.ctypes.data, u.ctypes.data))
        return rho, u

    def release(self, rid):
        _check(lib().lbmep_server_release(self._h, rid))
        self.meta.pop(rid, None)

    def stats(self):
        st = ServerStats()
        _check(lib().lbmep_server_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def now(self):
        t = np.zeros(1)
        _check(lib().lbmep_server_now(self._h, _dp(t)))
        return float(t[0])

    def wait_all(self, ids, timeout=600.0, sleep=5e-4):
        """Poll until every id in `ids` has finished; returns them in
        completion order."""
        import time
        pending = set(ids)
        order = []
        t0 = time.monotonic()
        while pending:
            for i in self.poll():
                if i in pending:
                    pending.discard(i)
                    order.append(i)
            if pending:
                if time.monotonic() - t0 > timeout:
                    raise TimeoutError(f"{len(pending)} requests still pending")
                time.sleep(sleep)
        return order
