"""ctypes binding of the plain FP64 CPU oracle (lbm_oracle.c).

TEST INFRASTRUCTURE ONLY: the checker of the GPU library.  Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import this module.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_oracle.so")
SRC = os.path.join(HERE, "lbm_oracle.c")

FLUID, WALL, OBST, NEAR = 0, 1, 2, 3

# D3Q19 ordering used by the oracle (q=0 rest, 1..6 axes, 7..18 diagonals)
C = np.array([
    [0, 0, 0],
    [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
    [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
    [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
    [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=np.int64)
W = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)


def build(force=True):
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-std=c99", "-Wall", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_create.restype = P
        L.orc_create.argtypes = [ctypes.c_int] * 3 + [ip, ctypes.c_double, ctypes.c_double]
        L.orc_destroy.argtypes = [P]
        L.orc_get_rates.argtypes = [P, dp]
        L.orc_set_flags.argtypes = [P, ctypes.c_void_p]
        L.orc_set_particles.argtypes = [P, ctypes.c_int, dp, dp, dp, dp, ctypes.c_int]
        L.orc_set_force.argtypes = [P, dp]
        L.orc_set_potential_force.argtypes = [P, dp, ctypes.c_double, dp, ctypes.c_void_p]
        L.orc_get_force.argtypes = [P, dp]
        L.orc_set_potential_solver.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                               ctypes.c_double, ctypes.c_int]
        L.orc_solve_potential.argtypes = [P, ip, dp, dp]
        L.orc_get_solver_stats.argtypes = [P, ip, dp, dp]
        L.orc_dha_residual.argtypes = [P]
        L.orc_dha_residual.restype = ctypes.c_double
        L.orc_get_potential.argtypes = [P, dp]
        L.orc_set_dynamics.argtypes = [P, ctypes.c_double, ctypes.c_void_p, dp]
        L.orc_set_free_slip.argtypes = [P, ip]
        L.orc_get_particles.argtypes = [P, dp, dp, dp]
        L.orc_init_equilibrium.argtypes = [P, ctypes.c_double, dp]
        L.orc_set_pdfs.argtypes = [P, dp]
        L.orc_get_pdfs.argtypes = [P, dp]
        L.orc_step.argtypes = [P, ctypes.c_int]
        L.orc_get_step.argtypes = [P]
        L.orc_get_step.restype = ctypes.c_long
        L.orc_get_macro.argtypes = [P, dp, dp]
        L.orc_get_ft.argtypes = [P, dp, dp]
        L.orc_get_map.argtypes = [P, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_get_invariants.argtypes = [P, dp]
        L.orc_get_bookkeeping.argtypes = [P, dp]
        L.orc_get_positions.argtypes = [P, dp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Oracle:
    """One lattice of the CPU oracle.  Arrays use (z, y, x) numpy order."""

    def __init__(self, shape, periodic=(True, True, True), nu=1.0 / 6.0, magic=3.0 / 16.0):
        self.shape = tuple(int(s) for s in shape)
        nx, ny, nz = self.shape
        self.N = nx * ny * nz
        per = (ctypes.c_int * 3)(*[1 if p else 0 for p in periodic])
        self._h = lib().orc_create(nx, ny, nz, per, float(nu), float(magic))
        if not self._h:
            raise ValueError("oracle: invalid lattice parameters")
        self.np = 0

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def rates(self):
        out = np.zeros(3)
        lib().orc_get_rates(self._h, _dp(out))
        return out

    def set_flags(self, flags):
        f = np.ascontiguousarray(flags, dtype=np.uint8).reshape(-1)
        assert f.size == self.N
        lib().orc_set_flags(self._h, f.ctypes.data)

    def set_particles(self, X, R, U, W=None, moving=False):
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 3)
        R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1)
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(-1, 3)
        n = len(R)
        Wa = np.zeros((n, 3)) if W is None else np.ascontiguousarray(W, dtype=np.float64).reshape(-1, 3)
        self.np = n
        self._keep = (X, R, U, Wa)
        lib().orc_set_particles(self._h, n, _dp(X), _dp(R), _dp(U), _dp(Wa), 1 if moving else 0)

    def set_force(self, fb):
        f = np.ascontiguousarray(fb, dtype=np.float64).reshape(-1)
        assert f.size == 3 * self.N
        lib().orc_set_force(self._h, _dp(f))

    def set_potential_force(self, psi, kappa2_eps, E, zeta=None):
        """Body force rho_e(psi) (E - grad psi) from the EDL potential psi
        (nz, ny, nx), rho_e = -kappa2_eps psi; zeta[np] = surface potential
        of each particle (None: the field's value at its obstacle cells)."""
        p = np.ascontiguousarray(psi, dtype=np.float64).reshape(-1)
        Ea = np.ascontiguousarray(E, dtype=np.float64)
        zp = None
        if zeta is not None:
            z = np.ascontiguousarray(zeta, dtype=np.float64).reshape(-1)
            self._zeta_keep = z
            zp = z.ctypes.data
        lib().orc_set_potential_force(self._h, _dp(p), float(kappa2_eps), _dp(Ea), zp)

    def set_potential_solver(self, kappa2, omega=1.7, max_iter=0, rf=0.0, check_every=1):
        """Red-black SOR for the Debye-Hueckel equation of the potential set
        by set_potential_force; max_iter > 0 also solves before every step."""
        rc = lib().orc_set_potential_solver(self._h, float(kappa2), float(omega), int(max_iter),
                                            float(rf), int(check_every))
        if rc:
            raise ValueError("oracle: bad solver parameters (odd periodic extent?)")

    def solve_potential(self):
        """One solve on the current map: (iterations, res0, res)."""
        it = ctypes.c_int(0)
        r0 = ctypes.c_double(0)
        r = ctypes.c_double(0)
        lib().orc_solve_potential(self._h, ctypes.byref(it), ctypes.byref(r0), ctypes.byref(r))
        return it.value, r0.value, r.value

    def solver_stats(self):
        it = ctypes.c_int(0)
        r0 = ctypes.c_double(0)
        r = ctypes.c_double(0)
        lib().orc_get_solver_stats(self._h, ctypes.byref(it), ctypes.byref(r0), ctypes.byref(r))
        return it.value, r0.value, r.value

    def dha_residual(self):
        return lib().orc_dha_residual(self._h)

    def potential(self):
        nx, ny, nz = self.shape
        out = np.zeros((nz, ny, nx))
        lib().orc_get_potential(self._h, _dp(out))
        return out

    def set_dynamics(self, rho_p, q=None, E=(0.0, 0.0, 0.0)):
        """Newton-Euler dynamics of the moving particles: density rho_p,
        charges q (None: 0), applied field E for the forces q E."""
        qp = None
        if q is not None:
            qa = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
            self._q_keep = qa
            qp = qa.ctypes.data
        Ea = np.ascontiguousarray(E, dtype=np.float64)
        if lib().orc_set_dynamics(self._h, float(rho_p), qp, _dp(Ea)):
            raise ValueError("oracle: dynamics need moving particles and rho_p > 0")

    def set_free_slip(self, faces):
        """Free-slip faces (x-, x+, y-, y+, z-, z+), non-periodic axes only."""
        f = (ctypes.c_int * 6)(*[1 if v else 0 for v in faces])
        if lib().orc_set_free_slip(self._h, f):
            raise ValueError("oracle: free-slip only on non-periodic axes")

    def particles(self):
        """Current positions, velocities and angular velocities (np, 3)."""
        X = np.zeros((self.np, 3))
        U = np.zeros((self.np, 3))
        Wv = np.zeros((self.np, 3))
        lib().orc_get_particles(self._h, _dp(X), _dp(U), _dp(Wv))
        return X, U, Wv

    def force(self):
        nx, ny, nz = self.shape
        fb = np.zeros((3, nz, ny, nx))
        lib().orc_get_force(self._h, _dp(fb))
        return fb

    def init_equilibrium(self, rho=1.0, u=(0.0, 0.0, 0.0)):
        ua = np.array(u, dtype=np.float64)
        lib().orc_init_equilibrium(self._h, float(rho), _dp(ua))

    def set_pdfs(self, f):
        a = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        assert a.size == 19 * self.N
        lib().orc_set_pdfs(self._h, _dp(a))

    def get_pdfs(self):
        nx, ny, nz = self.shape
        out = np.zeros((19, nz, ny, nx))
        lib().orc_get_pdfs(self._h, _dp(out))
        return out

    def step(self, n=1):
        lib().orc_step(self._h, int(n))

    @property
    def time(self):
        return lib().orc_get_step(self._h)

    def macro(self):
        nx, ny, nz = self.shape
        rho = np.zeros((nz, ny, nx))
        u = np.zeros((3, nz, ny, nx))
        lib().orc_get_macro(self._h, _dp(rho), _dp(u))
        return rho, u

    def ft(self):
        F = np.zeros((self.np, 3))
        M = np.zeros((self.np, 3))
        if self.np:
            lib().orc_get_ft(self._h, _dp(F), _dp(M))
        return F, M

    def map(self):
        nx, ny, nz = self.shape
        fl = np.zeros((nz, ny, nx), dtype=np.uint8)
        ow = np.zeros((nz, ny, nx), dtype=np.int32)
        lib().orc_get_map(self._h, fl.ctypes.data, ow.ctypes.data)
        return fl, ow

    def invariants(self):
        out = np.zeros(4)
        lib().orc_get_invariants(self._h, _dp(out))
        return out

    def bookkeeping(self):
        out = np.zeros(11)
        lib().orc_get_bookkeeping(self._h, _dp(out))
        return out

    def positions(self):
        X = np.zeros((self.np, 3))
        if self.np:
            lib().orc_get_positions(self._h, _dp(X))
        return X


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    lib().orc_set_num_threads(int(n))


def from_workload(wl):
    """Set up an oracle lattice for a workloads.Workload."""
    o = Oracle(wl.shape, wl.periodic, wl.nu, wl.magic)
    o.set_flags(wl.flags)
    o.set_force(wl.dense_force())
    o.init_equilibrium(1.0, (0.0, 0.0, 0.0))
    o.set_particles(wl.X, wl.R, wl.U, wl.W, wl.moving)
    return o
